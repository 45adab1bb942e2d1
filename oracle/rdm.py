"""Oracle reduced density matrices and gradients.  Test infrastructure only.

For a CASCI energy f(A) (lowest eigenvalue of the full-space Hamiltonian on
the determinant space of A), Hellmann-Feynman gives
  df/dh_pq = gamma_pq,   df/d(pq|rs) = 1/2 Gamma_pqrs,
with the full-space spin-summed RDMs computed in ``sc.c`` by applying every
operator string to every determinant.  For 8-fold symmetric integrals the
returned two-electron gradient is 1/2 Sym8(Gamma) (average over the eight
index permutations that leave (pq|rs) unchanged) and the one-electron one is
the symmetric part of gamma; contracted with any symmetric direction they
give the directional derivative.  Gradients of the expansion energy follow by
the chain rule through the Eq. 2 recursion (``mbe.increment_adjoint``).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _sc, fci, mbe


def rdm12(amasks, bmasks, c, norb):
    """Full-space spin-summed (gamma [M,M], Gamma [M,M,M,M]) of vector c."""
    L = _sc.lib()
    a = _sc.u64(amasks)
    b = _sc.u64(bmasks)
    c = _sc.f64(c)
    gamma = np.zeros((norb, norb))
    Gamma = np.zeros((norb,) * 4)
    dp = ctypes.c_double
    L.sc_rdm12(norb, len(a), _sc.ptr(a, ctypes.c_uint64), len(b), _sc.ptr(b, ctypes.c_uint64),
               _sc.ptr(c, dp), _sc.ptr(gamma, dp), _sc.ptr(Gamma, dp))
    return gamma, Gamma


def sym8(G):
    """Average of a 4-index array over the 8 permutations of (pq|rs)."""
    return (G + G.transpose(1, 0, 2, 3) + G.transpose(0, 1, 3, 2) + G.transpose(1, 0, 3, 2)
            + G.transpose(2, 3, 0, 1) + G.transpose(3, 2, 0, 1) + G.transpose(2, 3, 1, 0)
            + G.transpose(3, 2, 1, 0)) / 8.0


def casci_rdms(h, g, e_const, occ, active):
    """(energy, gamma, Gamma) of the CASCI ground state of ``active``."""
    a, b = fci.casci_space(occ, active)
    H = fci.hamiltonian(h, g, e_const, a, b)
    e, v = fci.lowest(H, want_vec=True)
    v = v / np.linalg.norm(v)
    gamma, Gamma = rdm12(a, b, v, h.shape[0])
    return e, gamma, Gamma


def casci_gradient(h, g, e_const, occ, active):
    """(f, df/dh, df/dg) of one CASCI, symmetrised as described above."""
    e, gamma, Gamma = casci_rdms(h, g, e_const, occ, active)
    return e, 0.5 * (gamma + gamma.T), 0.5 * sym8(Gamma)


def _grad_job(args):
    h, g, e_const, occ, active = args
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return casci_gradient(h, g, e_const, occ, active)
    except ImportError:  # pragma: no cover
        return casci_gradient(h, g, e_const, occ, active)


def mbe_gradient(prob, g_ref, g_order, workers=1):
    """d(g_ref E_ref + sum_n g_n E^(n)) / d(h, g) for a ``workloads.Problem``."""
    tups = mbe.tuples(prob.exp, prob.max_order)
    allt = [()] + tups
    jobs = [(prob.h1, prob.eri, prob.e_const, list(prob.occ), sorted(set(prob.ref) | set(t)))
            for t in allt]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_grad_job, jobs, chunksize=max(1, len(jobs) // (8 * workers))))
    else:
        res = [_grad_job(j) for j in jobs]
    f_ref = res[0][0]
    f = {t: r[0] for t, r in zip(tups, res[1:])}
    w_ref, w = mbe.increment_adjoint(g_ref, g_order, tups)
    dh = w_ref * res[0][1]
    dg = w_ref * res[0][2]
    for t, r in zip(tups, res[1:]):
        if w[t] != 0.0:
            dh = dh + w[t] * r[1]
            dg = dg + w[t] * r[2]
    return dh, dg, f_ref, f


def energy_from_rdms(h, g, e_const, gamma, Gamma):
    """E = sum h gamma + 1/2 sum (pq|rs) Gamma + e_const."""
    return float(np.sum(h * gamma) + 0.5 * np.sum(g * Gamma) + e_const)
