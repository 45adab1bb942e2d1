"""Seeded synthetic inputs for the generalized MBE-FCI hot path.

This module only *builds inputs*: molecular-orbital integrals h_pq and (pq|rs)
plus the orbital partition (occupied set O, reference space R, expansion space
X, maximum order).  It holds none of the method's arithmetic (no determinant,
CASCI or many-body-expansion code), so both the CPU oracle and the HIP path
can consume it without sharing any of the method.

Workloads (all FP64, chemist-order integrals, 0-based orbital indices):

* ``hubbard8``   -- 1D Hubbard, 8 sites, open, t=1, U=2, half filling, empty
  reference, full expansion to order 8 (the paper's Type-3 "vacuum"
  reference, Eq. 3).
* ``hubbard16``  -- 1D Hubbard, 16 sites, open, t=1, U=4, half filling; the
  reference space is the 6 MOs nearest the Fermi level, expansion over the
  other 10 MOs to order 4 (the paper's general reference/expansion split,
  Eq. 1).
* ``synthetic40`` -- molecular-like synthetic Hamiltonian, M=40, 12 electrons,
  (6e,6o) reference, order-3 expansion over 34 MOs.
* ``hubbard12``  -- 1D Hubbard, 12 sites, open, t=1, U=3, half filling, empty
  reference, order 6 (used for the gradient / backward path).
* ``cas14``      -- 8 synthetic CAS(14e,14o) instances, M=14, seeds 1..8, the
  whole space active (11,778,624 determinants each: the size of the paper's
  largest Hubbard CASCI).
* ``cas14_d2h``   -- 8 CAS(14e,14o) instances of the same size whose integrals
  respect D2h (``synthetic_sym``, two orbitals per irrep 0..6, seeds
  101..108), for the point-group blocked path.
* ``hubbardN_pm`` (``hubbardN_pm_uU``) -- 1D Hubbard, N sites, open, t=1, U=2
  (or U), half filling, in Pipek-Mezey localised orbitals: the paper's Type-3
  lattice runs (22, 34 and 46 sites, U/t <= 3), empty reference space, every
  MO in X, orders up to min(N, 14).

Localised orbitals: the occupied and the virtual hopping eigenvectors are
rotated separately (so the reference determinant, and its energy, stay the
same) to maximise the Pipek-Mezey locality sum_i sum_A (c_Ai^2)^2, the site
populations of an orthonormal site basis; then each block is ordered by
orbital centroid sum_A A c_Ai^2 and each orbital's largest coefficient made
positive.  The occupied block comes first.

Hubbard MOs are the eigenvectors of the open-chain hopping matrix in closed
form, phi_k(j) = sqrt(2/(N+1)) sin(pi j k/(N+1)), ordered by orbital energy
-2t cos(pi k/(N+1)); the on-site U tensor is transformed to that basis.  The
synthetic generator draws, from ``numpy.random.default_rng(seed)``: sorted
diagonal orbital energies ~ U(-2, 1); symmetric off-diagonal h_pq ~
N(0, 0.05 exp(-|p-q|/6)); 120 symmetric Cholesky-like vectors L^P with the same
decay; and (pq|rs) = sum_P L^P_pq L^P_rs, which is 8-fold symmetric.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import re

import numpy as np

__all__ = [
    "Problem",
    "hubbard_site",
    "hubbard_mo",
    "synthetic",
    "synthetic_sym",
    "pipek_mezey",
    "hubbard_pm",
    "lieb_wu_energy",
    "problem",
    "WORKLOADS",
    "checksum",
]


@dataclasses.dataclass
class Problem:
    """One MBE-FCI problem statement: integrals plus the orbital partition."""

    name: str
    h1: np.ndarray          # [M, M] symmetric
    eri: np.ndarray         # [M, M, M, M] chemist order (pq|rs)
    e_const: float
    occ: list               # doubly occupied orbitals of the reference determinant
    ref: list               # reference space R (possibly empty)
    exp: list               # expansion space X (disjoint from R)
    max_order: int
    orbsym: list = None     # point-group irrep label (0..7) per MO, or None

    @property
    def norb(self) -> int:
        return int(self.h1.shape[0])

    @property
    def nelec(self) -> int:
        return 2 * len(self.occ)


def hubbard_site(nsite: int, t: float, u: float):
    """Site-basis integrals of the open 1D Hubbard chain."""
    h = np.zeros((nsite, nsite))
    for j in range(nsite - 1):
        h[j, j + 1] = h[j + 1, j] = -t
    g = np.zeros((nsite,) * 4)
    for j in range(nsite):
        g[j, j, j, j] = u
    return h, g


def hubbard_orbitals(nsite: int):
    """Closed-form hopping eigenvectors: column k-1 is phi_k, k = 1..N."""
    j = np.arange(1, nsite + 1, dtype=np.float64)[:, None]
    k = np.arange(1, nsite + 1, dtype=np.float64)[None, :]
    return math.sqrt(2.0 / (nsite + 1)) * np.sin(np.pi * j * k / (nsite + 1))


def hubbard_mo(nsite: int, t: float, u: float):
    """Hubbard integrals in the hopping-eigenvector (MO) basis."""
    h_site, _ = hubbard_site(nsite, t, u)
    c = hubbard_orbitals(nsite)
    h = c.T @ h_site @ c
    h = 0.5 * (h + h.T)
    # (pq|rs) = U sum_j C_jp C_jq C_jr C_js
    pair = np.einsum("jp,jq->jpq", c, c).reshape(nsite, nsite * nsite)
    g = (u * pair.T @ pair).reshape((nsite,) * 4)
    return h, g


def pipek_mezey(c: np.ndarray, tol: float = 1e-13, max_sweeps: int = 5000) -> np.ndarray:
    """Pipek-Mezey localisation of the orthonormal columns of ``c`` (rows: an
    orthonormal site basis, so column i has population c[A, i]^2 on site A).

    Maximises L = sum_i sum_A c[A, i]^4 by Jacobi sweeps over column pairs.
    Rotating the pair (x, y) -> (cos g x + sin g y, -sin g x + cos g y) changes
    L by P (1 - cos 4g) + Q sin 4g, with P = sum_A [(x y)^2 - (x^2 - y^2)^2 / 4]
    and Q = sum_A x y (x^2 - y^2); the best angle has (cos 4g, sin 4g)
    proportional to (-P, Q) and gains P + sqrt(P^2 + Q^2) >= 0.  Sweeps stop
    when no pair gains more than ``tol``.
    """
    c = np.array(c, dtype=np.float64, copy=True)
    n = c.shape[1]
    for _ in range(max_sweeps):
        best = 0.0
        for s in range(n):
            for t in range(s + 1, n):
                x, y = c[:, s].copy(), c[:, t].copy()
                xy = x * y
                d = x * x - y * y
                p = float(np.sum(xy * xy - 0.25 * d * d))
                q = float(np.sum(d * xy))
                gain = p + math.hypot(p, q)
                if gain > tol:
                    g = 0.25 * math.atan2(q, -p)
                    cs, sn = math.cos(g), math.sin(g)
                    c[:, s] = cs * x + sn * y
                    c[:, t] = -sn * x + cs * y
                    best = max(best, gain)
        if best <= tol:
            return c
    raise RuntimeError("Pipek-Mezey sweeps did not converge")


def _order_and_sign(c: np.ndarray) -> np.ndarray:
    sites = np.arange(c.shape[0], dtype=np.float64)
    cen = sites @ (c * c)
    c = c[:, np.argsort(cen, kind="stable")]
    big = np.argmax(np.abs(c), axis=0)
    sign = np.sign(c[big, np.arange(c.shape[1])])
    return c * sign


def hubbard_pm(nsite: int, t: float, u: float):
    """Hubbard integrals in Pipek-Mezey localised orbitals (occupied block
    first, see the module docstring); returns (h, g, C) with C the site x
    orbital coefficients."""
    if nsite % 2:
        raise ValueError("half filling needs an even number of sites")
    h_site, _ = hubbard_site(nsite, t, u)
    c0 = hubbard_orbitals(nsite)
    nocc = nsite // 2
    c = np.hstack([_order_and_sign(pipek_mezey(c0[:, :nocc])),
                   _order_and_sign(pipek_mezey(c0[:, nocc:]))])
    h = c.T @ h_site @ c
    h = 0.5 * (h + h.T)
    pair = np.einsum("jp,jq->jpq", c, c).reshape(nsite, nsite * nsite)
    g = (u * pair.T @ pair).reshape((nsite,) * 4)
    return h, g, c


def lieb_wu_energy(u: float, t: float = 1.0) -> float:
    """Ground-state energy per site of the half-filled 1D Hubbard model in the
    thermodynamic limit (Lieb and Wu, 1968):
    E/N = -4t int_0^inf J0(w) J1(w) / (w (1 + exp(w U / 2t))) dw.
    A reference value for the lattice workloads (open chains of N sites lie
    above it by a boundary term of order 1/N), not part of the expansion.
    """
    from scipy import integrate, special

    def f(w):
        return special.j0(w) * special.j1(w) / w * special.expit(-w * u / (2.0 * t))

    wmax = 4000.0 if u <= 0 else min(4000.0, 90.0 * t / u + 40.0)
    edges = np.arange(0.0, wmax + math.pi, math.pi)
    val = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        val += integrate.quad(f, lo, hi, limit=100, epsabs=1e-14, epsrel=1e-12)[0]
    return -4.0 * t * val


def synthetic(norb: int, seed: int, nchol: int = 120):
    """Molecular-like synthetic integrals (see module docstring)."""
    rng = np.random.default_rng(seed)
    h = np.zeros((norb, norb))
    h[np.diag_indices(norb)] = np.sort(rng.uniform(-2.0, 1.0, norb))
    iu = np.triu_indices(norb, 1)
    sd = 0.05 * np.exp(-np.abs(iu[0] - iu[1]) / 6.0)
    off = rng.standard_normal(len(sd)) * sd
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(norb, 0)
    sd0 = 0.05 * np.exp(-np.abs(iu0[0] - iu0[1]) / 6.0)
    lmat = np.zeros((nchol, norb, norb))
    for p in range(nchol):
        v = rng.standard_normal(len(sd0)) * sd0
        lmat[p][iu0] = v
        lmat[p][(iu0[1], iu0[0])] = v
    flat = lmat.reshape(nchol, norb * norb)
    g = (flat.T @ flat).reshape((norb,) * 4)
    return h, g


def synthetic_sym(norb: int, seed: int, orbsym, nchol: int = 120):
    """Synthetic integrals that respect a point group with abelian irreps
    labelled 0..7 (D2h and its subgroups; the product of two irreps is the
    XOR of their labels): the same distributions as ``synthetic``, with h_pq
    kept only where orbsym[p] == orbsym[q], and Cholesky-like vectors L^P of
    irrep P % 8 kept only where orbsym[p] ^ orbsym[q] == P % 8, so that
    (pq|rs) = sum_P L^P_pq L^P_rs vanishes unless the four irreps multiply to
    the totally symmetric one.  ``orbsym``: [norb] labels 0..7."""
    sym = np.asarray(orbsym, dtype=np.int64)
    if sym.shape != (norb,) or np.any(sym < 0) or np.any(sym > 7):
        raise ValueError("orbsym must hold norb labels in 0..7")
    h, _ = synthetic(norb, seed, nchol=1)
    h = np.where(sym[:, None] == sym[None, :], h, 0.0)
    rng = np.random.default_rng(seed + 7919)
    iu0 = np.triu_indices(norb, 0)
    sd0 = 0.05 * np.exp(-np.abs(iu0[0] - iu0[1]) / 6.0)
    pair_sym = sym[iu0[0]] ^ sym[iu0[1]]
    lmat = np.zeros((nchol, norb, norb))
    for p in range(nchol):
        v = rng.standard_normal(len(sd0)) * sd0 * (pair_sym == p % 8)
        lmat[p][iu0] = v
        lmat[p][(iu0[1], iu0[0])] = v
    flat = lmat.reshape(nchol, norb * norb)
    g = (flat.T @ flat).reshape((norb,) * 4)
    return h, g


def _hubbard_problem(name, nsite, u, ref, max_order):
    h, g = hubbard_mo(nsite, 1.0, u)
    occ = list(range(nsite // 2))
    exp = [p for p in range(nsite) if p not in ref]
    return Problem(name, h, g, 0.0, occ, list(ref), exp, max_order)


def problem(name: str, instance: int = 0) -> Problem:
    """Build one named workload (``instance`` selects the cas14 seed 1..8)."""
    if name == "hubbard8":
        return _hubbard_problem(name, 8, 2.0, [], 8)
    if name == "hubbard16":
        # 1-based MOs k = 6..11 are the 3 occupied + 3 virtual nearest the Fermi level
        return _hubbard_problem(name, 16, 4.0, list(range(5, 11)), 4)
    if name == "hubbard12":
        return _hubbard_problem(name, 12, 3.0, [], 6)
    if name == "hubbard16_vacuum":
        # the paper's Type-3 setting: empty reference space, every MO in X;
        # order-by-order with screening (orders 2..8)
        return _hubbard_problem(name, 16, 4.0, [], 8)
    if name == "synthetic40":
        h, g = synthetic(40, 0)
        occ = list(range(6))
        ref = list(range(3, 9))
        exp = [p for p in range(40) if p not in ref]
        return Problem(name, h, g, 0.0, occ, ref, exp, 3)
    if name == "cas14":
        if not 0 <= instance < 8:
            raise ValueError("cas14 has instances 0..7 (seeds 1..8)")
        h, g = synthetic(14, instance + 1)
        occ = list(range(7))
        return Problem(f"cas14[{instance}]", h, g, 0.0, occ, list(range(14)), [], 0)
    if name == "cas14_d2h":
        # the same size with D2h-symmetric integrals: two orbitals per irrep
        # (irreps 0..6), seeds 101..108
        if not 0 <= instance < 8:
            raise ValueError("cas14_d2h has instances 0..7 (seeds 101..108)")
        osym = [p // 2 for p in range(14)]
        h, g = synthetic_sym(14, 101 + instance, osym)
        return Problem(f"cas14_d2h[{instance}]", h, g, 0.0, list(range(7)), list(range(14)), [],
                       0, orbsym=osym)
    pm = re.fullmatch(r"hubbard(\d+)_pm(?:_u(\d+(?:\.\d+)?))?", name)
    if pm:
        n = int(pm.group(1))
        u = float(pm.group(2)) if pm.group(2) else 2.0
        h, g, _ = hubbard_pm(n, 1.0, u)
        return Problem(name, h, g, 0.0, list(range(n // 2)), [], list(range(n)), min(n, 14))
    if name.startswith("hubbard") and name[7:].isdigit():
        n = int(name[7:])
        return _hubbard_problem(name, n, 2.0, [], n)
    raise KeyError(name)


WORKLOADS = ("hubbard8", "hubbard16", "synthetic40", "hubbard12", "cas14")


def checksum(*arrays) -> str:
    """SHA-256 over the raw little-endian bytes of the given arrays."""
    m = hashlib.sha256()
    for a in arrays:
        m.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return m.hexdigest()
