"""Pins of the point-group oracle (``oracle/sym.py``) and the symmetric
synthetic generator (``workloads.synthetic_sym``).

* The generator's integrals vanish exactly where the point group says they
  must: h_pq unless irr(p) = irr(q), (pq|rs) unless the four irreps XOR to 0.
* With such integrals the Slater-Condon Hamiltonian couples no two irreps
  (every CSR element between different sectors is zero), the sectors
  partition the determinant space, and the union of the eight sectors'
  spectra is the whole spectrum (dense diagonalisation, frozen core and
  unequal spins included).
* Sector dimensions from string counts per irrep equal brute-force counts,
  and the paper's Cr2 size: a CAS(16e,16o) with two orbitals per D2h irrep
  has 20,708,900 totally symmetric determinants, the 2.07e7 the Cr2
  discussion (Fig. 3) quotes "with D2h symmetry".
* The MBE with every CASCI in the totally symmetric irrep telescopes at full
  order to the whole space's totally symmetric FCI energy.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import fci, mbe, sym

ORBSYM8 = [0, 5, 3, 6, 0, 1, 7, 2]


def test_generator_respects_the_point_group():
    h, g = W.synthetic_sym(8, 3, ORBSYM8)
    s = np.array(ORBSYM8)
    assert np.all(h[s[:, None] != s[None, :]] == 0.0)
    assert np.any(h[s[:, None] == s[None, :]] != 0.0)
    x = s[:, None, None, None] ^ s[None, :, None, None] ^ s[None, None, :, None] ^ s[None, None, None, :]
    assert np.all(g[x != 0] == 0.0)
    assert np.count_nonzero(g[x == 0]) > 0.5 * np.count_nonzero(x == 0)
    assert np.allclose(g, g.transpose(1, 0, 2, 3)) and np.allclose(g, g.transpose(2, 3, 0, 1))


@pytest.mark.parametrize("occ,active,na,nb", [
    ([0, 1, 2], list(range(6)), None, None),
    ([0, 1, 2, 3], [1, 2, 3, 4, 5, 6], None, None),  # 0 frozen, 7 deleted
    (None, list(range(6)), 3, 2),                      # unequal spins
])
def test_sectors_partition_the_spectrum(occ, active, na, nb):
    h, g = W.synthetic_sym(8, 5, ORBSYM8)
    if occ is not None:
        a, b = fci.casci_space(occ, active)
    else:
        a, b = fci.string_masks(active, na), fci.string_masks(active, nb)
    H = fci.hamiltonian(h, g, 0.1, a, b)
    n = H.shape[0]
    idx = [sym.sector(a, b, ORBSYM8, G) for G in range(8)]
    allidx = np.sort(np.concatenate(idx))
    assert np.array_equal(allidx, np.arange(n))
    Hd = H.toarray()
    for G in range(8):
        for Gp in range(8):
            if G != Gp and len(idx[G]) and len(idx[Gp]):
                assert np.all(Hd[np.ix_(idx[G], idx[Gp])] == 0.0)
    full = scipy.linalg.eigvalsh(Hd)
    parts = np.sort(np.concatenate([scipy.linalg.eigvalsh(Hd[np.ix_(i, i)]) for i in idx if len(i)]))
    assert np.max(np.abs(full - parts)) < 1e-10
    # the lowest sector energy is the unblocked lowest eigenvalue
    lows = []
    for G in range(8):
        Hs, _ = sym.hamiltonian(h, g, 0.1, a, b, ORBSYM8, G)
        if Hs.shape[0]:
            lows.append(fci.lowest(Hs))
    assert abs(min(lows) - full[0]) < 1e-10


def test_sector_dims_against_brute_force():
    act = list(range(7))
    osym = [1, 4, 4, 7, 0, 2, 3]
    dims = sym.sector_dims(7, 3, 4, osym)
    a, b = fci.string_masks(act, 3), fci.string_masks(act, 4)
    for G in range(8):
        assert dims[G] == len(sym.sector(a, b, osym, G))
    assert sum(dims) == len(a) * len(b)


def test_paper_cr2_d2h_casci_size():
    """CAS(16e,16o), two orbitals per D2h irrep, totally symmetric sector."""
    dims = sym.sector_dims(16, 8, 8, [p // 2 for p in range(16)])
    assert dims[0] == 20708900
    assert round(dims[0] / 1e7, 2) == 2.07


def test_full_order_mbe_in_the_symmetric_irrep_equals_fci():
    h, g = W.synthetic_sym(7, 11, ORBSYM8[:7])
    p = W.Problem("sym7", h, g, 0.0, [0, 1, 2], [], list(range(7)), 7, orbsym=ORBSYM8[:7])
    r = mbe.mbe(p, workers=4)
    exact = sym.casci(h, g, 0.0, p.occ, range(7), ORBSYM8[:7], 0)
    assert abs(r["e_total"] - exact) < 1e-10
    # vacuum reference (Eq. 3): order 1 vanishes
    assert abs(r["e_order"][0]) < 1e-12
