"""Pins of the matrix-free oracle CASCI (``oracle/direct.py``, the
``sc_direct_*`` functions of ``oracle/sc.c``).

* sigma = H c element by element against the stored Slater-Condon CSR
  Hamiltonian (``fci.hamiltonian``, itself pinned against second-quantised
  brute force) on spaces with every kind of excitation: whole active
  spaces, frozen doubly occupied and deleted orbitals, unequal alpha and beta
  electron counts, one-electron strings, and single-determinant spaces.
* Row splits over threads do not change sigma (each row is summed by one
  thread in a fixed order): bitwise equal.
* Lowest eigenvalue by Lanczos on the operator against the oracle's dense /
  CSR eigensolver, and the two-site Hubbard closed form
  E = (U - sqrt(U^2 + 16 t^2)) / 2.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct, fci

CASES = [
    # (M, seed, occ, active, nalpha override, nbeta override)
    (6, 7, [0, 1, 2], list(range(6)), None, None),
    (8, 7, [0, 1, 2], [1, 2, 4, 5, 6], None, None),      # 0 frozen, 3 and 7 deleted
    (7, 9, [0, 1, 2, 3], [0, 2, 3, 4, 5, 6], None, None),  # 1 frozen
    (6, 3, None, list(range(6)), 3, 2),                   # unbalanced spins
    (5, 4, None, list(range(5)), 1, 4),                   # one alpha electron
    (4, 5, [0, 1], [0, 1], None, None),                   # a single determinant
]


def _space(M, occ, active, na, nb):
    if na is None:
        return fci.casci_space(occ, active)
    return fci.string_masks(active, na), fci.string_masks(active, nb)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sigma_matches_stored_hamiltonian(case):
    M, seed, occ, active, na, nb = CASES[case]
    h, g = W.synthetic(M, seed)
    a, b = _space(M, occ, active, na, nb)
    Hs = fci.hamiltonian(h, g, 0.37, a, b)
    D = direct.DirectHamiltonian(h, g, 0.37, a, b, threads=3)
    try:
        rng = np.random.default_rng(seed)
        for _ in range(3):
            c = rng.standard_normal(Hs.shape[0])
            ref = Hs @ c
            got = D.matvec(c)
            assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
        # unit vectors: columns of H, diagonal included
        for j in rng.choice(Hs.shape[0], size=min(5, Hs.shape[0]), replace=False):
            e = np.zeros(Hs.shape[0])
            e[j] = 1.0
            assert np.max(np.abs(D.matvec(e) - Hs[:, j].toarray().ravel())) <= 1e-12
    finally:
        D.close()


def test_row_split_is_bitwise_neutral():
    h, g = W.synthetic(8, 11)
    a, b = fci.casci_space(range(4), range(8))
    c = np.random.default_rng(1).standard_normal(len(a) * len(b))
    outs = []
    for threads in (1, 3, 8):
        D = direct.DirectHamiltonian(h, g, 0.0, a, b, threads=threads)
        outs.append(D.matvec(c))
        D.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("name,occ,active", [
    ("hubbard8", [0, 1, 2, 3], list(range(8))),     # 4,900 determinants
    ("synth10", [0, 1, 2, 3, 4], [2, 3, 4, 5, 6, 7]),  # frozen 0, 1; deleted 8, 9
])
def test_lanczos_lowest_matches_oracle_eigensolver(name, occ, active):
    if name == "hubbard8":
        h, g = W.hubbard_mo(8, 1.0, 2.0)
    else:
        h, g = W.synthetic(10, 5)
    ref = fci.casci(h, g, 0.0, occ, active)
    got = direct.casci(h, g, 0.0, occ, active, threads=4)
    assert abs(got - ref) < 1e-10


def test_two_site_hubbard_closed_form():
    t, u = 1.0, 2.0
    h, g = W.hubbard_site(2, t, u)
    got = direct.casci(h, g, 0.0, [0], [0, 1], threads=1)
    assert abs(got - (u - math.sqrt(u * u + 16 * t * t)) / 2) < 1e-12
