"""Oracle CASCI: lowest eigenvalue of the Slater-Condon Hamiltonian on a
frozen-core determinant space.  Test infrastructure only.

For an active set A (sorted spatial orbitals) and the reference-determinant
occupied set O, the CASCI space D(A) holds every determinant whose alpha and
beta strings contain all of F = O \\ A (frozen, doubly occupied), none of the
orbitals outside A u O (deleted) and exactly |O n A| electrons of A.  This is
the reading under which the zero-increment rule stated with Eq. 3 holds.  H is
the full-space Hamiltonian (all M orbitals, frozen ones explicit) restricted
to D(A); its lowest eigenvalue is f(A) (the "CASCI energy" of Eq. 1 / Eq. 2).
"""
from __future__ import annotations

import ctypes
import itertools

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from . import _sc

DENSE_MAX = 2500  # dense eigh up to this many determinants, Lanczos above


def string_masks(active, nelec, frozen=()):
    """All strings with the frozen orbitals set and ``nelec`` electrons in
    ``active``, as full-space bitmasks in ascending integer order."""
    base = 0
    for f in frozen:
        base |= 1 << int(f)
    masks = []
    for comb in itertools.combinations(sorted(int(a) for a in active), nelec):
        m = base
        for o in comb:
            m |= 1 << o
        masks.append(m)
    return np.array(sorted(masks), dtype=np.uint64)


def casci_space(occ, active):
    """(alpha masks, beta masks) of the CASCI space of ``active`` (closed-shell
    reference determinant with doubly occupied orbitals ``occ``)."""
    occ = set(int(o) for o in occ)
    act = sorted(set(int(a) for a in active))
    frozen = sorted(occ - set(act))
    nel = len(occ & set(act))
    s = string_masks(act, nel, frozen)
    return s, s.copy()


def hamiltonian(h, g, e_const, amasks, bmasks):
    """Sparse CSR Hamiltonian over the product space (index ia*nb + ib)."""
    L = _sc.lib()
    h = _sc.f64(h)
    g = _sc.f64(g)
    M = h.shape[0]
    a = _sc.u64(amasks)
    b = _sc.u64(bmasks)
    dp = ctypes.c_double
    null64 = ctypes.POINTER(ctypes.c_int64)()
    null32 = ctypes.POINTER(ctypes.c_int32)()
    nulld = ctypes.POINTER(ctypes.c_double)()
    nnz = L.sc_build_csr(M, _sc.ptr(h, dp), _sc.ptr(g, dp), float(e_const), len(a),
                         _sc.ptr(a, ctypes.c_uint64), len(b), _sc.ptr(b, ctypes.c_uint64),
                         null64, null32, nulld)
    n = len(a) * len(b)
    indptr = np.zeros(n + 1, dtype=np.int64)
    indices = np.zeros(nnz, dtype=np.int32)
    data = np.zeros(nnz, dtype=np.float64)
    L.sc_build_csr(M, _sc.ptr(h, dp), _sc.ptr(g, dp), float(e_const), len(a),
                   _sc.ptr(a, ctypes.c_uint64), len(b), _sc.ptr(b, ctypes.c_uint64),
                   _sc.ptr(indptr, ctypes.c_int64), _sc.ptr(indices, ctypes.c_int32),
                   _sc.ptr(data, dp))
    return scipy.sparse.csr_matrix((data, indices, indptr), shape=(n, n))


def diagonal(h, g, e_const, amasks, bmasks):
    L = _sc.lib()
    h = _sc.f64(h)
    g = _sc.f64(g)
    a = _sc.u64(amasks)
    b = _sc.u64(bmasks)
    out = np.zeros(len(a) * len(b))
    dp = ctypes.c_double
    L.sc_diagonal(h.shape[0], _sc.ptr(h, dp), _sc.ptr(g, dp), float(e_const), len(a),
                  _sc.ptr(a, ctypes.c_uint64), len(b), _sc.ptr(b, ctypes.c_uint64),
                  _sc.ptr(out, dp))
    return out


def element(h, g, I, J):
    """<I|H|J> for full-space determinants I = (alpha mask, beta mask)."""
    h = _sc.f64(h)
    g = _sc.f64(g)
    dp = ctypes.c_double
    return _sc.lib().sc_element(h.shape[0], _sc.ptr(h, dp), _sc.ptr(g, dp),
                                int(I[0]), int(I[1]), int(J[0]), int(J[1]))


def sigma_rows(h, g, e_const, amasks, bmasks, c, rows):
    """sigma_I = (H c)_I for sampled product-space rows I, without forming H."""
    L = _sc.lib()
    h = _sc.f64(h)
    g = _sc.f64(g)
    a = _sc.u64(amasks)
    b = _sc.u64(bmasks)
    c = _sc.f64(c)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(len(rows))
    dp = ctypes.c_double
    L.sc_sigma_rows(h.shape[0], _sc.ptr(h, dp), _sc.ptr(g, dp), float(e_const), len(a),
                    _sc.ptr(a, ctypes.c_uint64), len(b), _sc.ptr(b, ctypes.c_uint64),
                    _sc.ptr(c, dp), len(rows), _sc.ptr(rows, ctypes.c_int64), _sc.ptr(out, dp))
    return out


def lowest(H, want_vec=False, tol=1e-13):
    """Lowest eigenpair of a real symmetric (sparse) matrix: dense ``eigh`` on
    small spaces, ARPACK Lanczos (``eigsh``, smallest algebraic) above."""
    n = H.shape[0]
    if n <= DENSE_MAX:
        w, v = scipy.linalg.eigh(H.toarray(), subset_by_index=[0, 0])
        return (w[0], v[:, 0]) if want_vec else w[0]
    # deterministic start vector with components in every symmetry sector
    v0 = np.cos(np.arange(n) * 0.7548776662466927) + 1.0
    w, v = scipy.sparse.linalg.eigsh(H, k=1, which="SA", tol=tol, v0=v0,
                                     ncv=min(n, 40), maxiter=100000)
    return (w[0], v[:, 0]) if want_vec else w[0]


def casci(h, g, e_const, occ, active, want_vec=False):
    """f(A): lowest eigenvalue (and eigenvector in the product-space basis of
    ``casci_space``) of H restricted to the CASCI space of ``active``."""
    a, b = casci_space(occ, active)
    H = hamiltonian(h, g, e_const, a, b)
    return lowest(H, want_vec)
