"""Matrix-free oracle CASCI for spaces too large for a stored Hamiltonian
(CAS(14,14): 11,778,624 determinants).  Test infrastructure only.

sigma = H c is formed row by row from Slater-Condon elements of the
determinants within two electrons of each row (``sc_direct_sigma`` in
``sc.c``), never storing H; the diagonal comes from ``sc_diagonal``.  Rows
are split over host threads (the C call releases the GIL).  The lowest
eigenvalue is found by ARPACK's implicitly restarted Lanczos (SciPy
``eigsh``) on that operator.  Pinned against the stored CSR Hamiltonian of
``fci.hamiltonian`` on small spaces (sigma element by element, and the
lowest eigenvalue).
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.sparse.linalg

from . import _sc, fci


class DirectHamiltonian:
    """H restricted to the product space of ``amasks`` x ``bmasks`` (full-space
    string bitmasks, ascending), applied without storing it."""

    def __init__(self, h, g, e_const, amasks, bmasks, threads=None):
        L = _sc.lib()
        self._L = L
        self.h = _sc.f64(h)
        self.g = _sc.f64(g)
        self.a = _sc.u64(amasks)
        self.b = _sc.u64(bmasks)
        self.na, self.nb = len(self.a), len(self.b)
        self.n = self.na * self.nb
        self.diag = fci.diagonal(self.h, self.g, e_const, self.a, self.b)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        M = self.h.shape[0]
        self._t = L.sc_direct_setup(M, _sc.ptr(self.h, ctypes.c_double),
                                    _sc.ptr(self.g, ctypes.c_double), self.na,
                                    _sc.ptr(self.a, ctypes.c_uint64), self.nb,
                                    _sc.ptr(self.b, ctypes.c_uint64),
                                    _sc.ptr(self.diag, ctypes.c_double))
        if not self._t:
            raise MemoryError("sc_direct_setup: out of memory")
        self.threads = threads or os.cpu_count() or 1
        self._pool = ThreadPoolExecutor(self.threads) if self.threads > 1 else None
        self.nmatvec = 0
        del dp, up

    def close(self):
        if self._t:
            self._L.sc_direct_free(self._t)
            self._t = None
        if self._pool:
            self._pool.shutdown()
            self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, c):
        c = _sc.f64(np.asarray(c).reshape(-1))
        out = np.empty(self.n)
        pc = _sc.ptr(c, ctypes.c_double)
        po = _sc.ptr(out, ctypes.c_double)
        if self._pool is None:
            self._L.sc_direct_sigma(self._t, pc, po, 0, self.na)
        else:
            # many more row blocks than threads: rows cost about the same
            nblk = min(self.na, 8 * self.threads)
            edges = np.linspace(0, self.na, nblk + 1).astype(int)
            jobs = [self._pool.submit(self._L.sc_direct_sigma, self._t, pc, po, int(lo), int(hi))
                    for lo, hi in zip(edges[:-1], edges[1:]) if hi > lo]
            for j in jobs:
                j.result()
        self.nmatvec += 1
        return out

    def operator(self):
        return scipy.sparse.linalg.LinearOperator((self.n, self.n), matvec=self.matvec,
                                                  dtype=np.float64)


def lowest(H: DirectHamiltonian, tol=1e-13, ncv=30, want_vec=False):
    """Lowest eigenpair by ARPACK Lanczos (smallest algebraic), from the same
    deterministic start vector as ``fci.lowest``."""
    n = H.n
    if n == 1:
        return (H.diag[0], np.ones(1)) if want_vec else H.diag[0]
    v0 = np.cos(np.arange(n) * 0.7548776662466927) + 1.0
    w, v = scipy.sparse.linalg.eigsh(H.operator(), k=1, which="SA", tol=tol, v0=v0,
                                     ncv=min(n - 1, ncv), maxiter=100000)
    return (w[0], v[:, 0]) if want_vec else w[0]


def casci(h, g, e_const, occ, active, tol=1e-13, threads=None, want_vec=False):
    """f(A) of the CASCI of ``active`` (frozen-core reading as in ``fci``)
    by the matrix-free operator."""
    a, b = fci.casci_space(occ, active)
    H = DirectHamiltonian(h, g, e_const, a, b, threads)
    try:
        return lowest(H, tol=tol, want_vec=want_vec)
    finally:
        H.close()
