"""Oracle CASCI in one irreducible representation of an abelian point group
(D2h and its subgroups).  Test infrastructure only.

The paper's Cr2 expansion solves its CASCIs with D2h symmetry (the Fig. 3
discussion quotes the largest as 2.07e7 determinants "with D2h symmetry").
Orbital irreps are labels 0..7 whose product is their XOR.  A determinant's
irrep is the XOR of the irreps of its occupied spin orbitals (alpha and
beta); doubly occupied orbitals cancel, so the frozen core and the
closed-shell reference determinant are totally symmetric (label 0).

The CASCI of irrep G keeps the determinants of the frozen-core space of
``fci.casci_space`` whose irrep is G and diagonalises the Slater-Condon
Hamiltonian restricted to them: the product-space CSR matrix of
``fci.hamiltonian`` with every row and column of another irrep dropped.
Nothing else changes; with integrals that respect the symmetry, H couples no
two irreps, so the union of the sectors' spectra is the whole spectrum
(pinned).
"""
from __future__ import annotations

import numpy as np

from . import fci


def string_irrep(mask, orbsym):
    """XOR of the irreps of the orbitals set in ``mask``."""
    s = 0
    m = int(mask)
    p = 0
    while m:
        if m & 1:
            s ^= int(orbsym[p])
        m >>= 1
        p += 1
    return s


def sector(amasks, bmasks, orbsym, irrep):
    """Product-space indices ia * nb + ib (ascending) of the determinants of
    irrep ``irrep``."""
    sa = np.array([string_irrep(m, orbsym) for m in amasks], dtype=np.int64)
    sb = np.array([string_irrep(m, orbsym) for m in bmasks], dtype=np.int64)
    keep = (sa[:, None] ^ sb[None, :]) == int(irrep)
    return np.flatnonzero(keep.ravel())


def hamiltonian(h, g, e_const, amasks, bmasks, orbsym, irrep):
    """(H restricted to the sector, the sector's product-space indices)."""
    H = fci.hamiltonian(h, g, e_const, amasks, bmasks)
    idx = sector(amasks, bmasks, orbsym, irrep)
    return H[idx][:, idx].tocsr(), idx


def casci(h, g, e_const, occ, active, orbsym, irrep=0, want_vec=False):
    """Lowest eigenvalue (and eigenvector over the sector's determinants, in
    the order of ``sector``) of the CASCI of ``active`` in irrep ``irrep``."""
    a, b = fci.casci_space(occ, active)
    H, _ = hamiltonian(h, g, e_const, a, b, orbsym, irrep)
    if H.shape[0] == 0:
        raise ValueError("no determinant of that irrep in this CASCI space")
    return fci.lowest(H, want_vec)


def sector_dims(norb_active, nalpha, nbeta, orbsym_active):
    """Dimension of every irrep's sector of the (nalpha, nbeta) space of the
    active orbitals: sum over alpha irreps a of N_alpha(a) N_beta(a ^ G)."""
    import itertools
    na = np.zeros(8, dtype=np.int64)
    nb = np.zeros(8, dtype=np.int64)
    for comb in itertools.combinations(range(norb_active), nalpha):
        s = 0
        for p in comb:
            s ^= int(orbsym_active[p])
        na[s] += 1
    for comb in itertools.combinations(range(norb_active), nbeta):
        s = 0
        for p in comb:
            s ^= int(orbsym_active[p])
        nb[s] += 1
    return [int(sum(na[a] * nb[a ^ G] for a in range(8))) for G in range(8)]
