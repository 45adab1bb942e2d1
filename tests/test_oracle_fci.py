"""Pins of the oracle's Slater-Condon CASCI against definitions, closed forms
and brute force (CPU only)."""
import itertools
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fci, strings as ostr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


def _random_integrals(M, seed):
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((M, M))
    h = 0.5 * (h + h.T)
    L = rng.standard_normal((5, M, M))
    L = 0.5 * (L + L.transpose(0, 2, 1))
    g = np.einsum("Ppq,Prs->pqrs", L, L)
    return h, g


# ---------------------------------------------------------------- brute force
def _so_apply(ops, det, M):
    """Apply a list of (kind, spin-orbital) right-to-left to a determinant given
    as a tuple of 2M occupations; returns (sign, det) or (0, None)."""
    occ = list(det)
    sign = 1
    for kind, P in reversed(ops):
        below = sum(occ[:P])
        if kind == "a":
            if not occ[P]:
                return 0, None
            occ[P] = 0
        else:
            if occ[P]:
                return 0, None
            occ[P] = 1
        if below % 2:
            sign = -sign
    return sign, tuple(occ)


def _brute_hamiltonian(h, g, dets, M):
    """H_IJ from the second-quantised Hamiltonian, operator by operator."""
    idx = {d: i for i, d in enumerate(dets)}
    n = len(dets)
    H = np.zeros((n, n))
    so = range(2 * M)

    def hs(P, Q):
        return h[P % M, Q % M] if P // M == Q // M else 0.0

    def gs(P, Q, R, S):
        if P // M != Q // M or R // M != S // M:
            return 0.0
        return g[P % M, Q % M, R % M, S % M]

    for j, d in enumerate(dets):
        for P in so:
            for Q in so:
                v = hs(P, Q)
                if v == 0.0:
                    continue
                s, r = _so_apply([("c", P), ("a", Q)], d, M)
                if s and r in idx:
                    H[idx[r], j] += s * v
        for P, Q, R, S in itertools.product(so, repeat=4):
            v = gs(P, Q, R, S)
            if v == 0.0:
                continue
            s, r = _so_apply([("c", P), ("c", R), ("a", S), ("a", Q)], d, M)
            if s and r in idx:
                H[idx[r], j] += 0.5 * s * v
    return H


@pytest.mark.parametrize("M,nel,seed", [(3, 1, 0), (3, 2, 1), (4, 2, 2), (4, 1, 3)])
def test_slater_condon_matches_second_quantisation(M, nel, seed):
    h, g = _random_integrals(M, seed)
    s = ostr.strings(M, nel)
    dets = []
    for a in s:
        for b in s:
            dets.append(tuple([(a >> p) & 1 for p in range(M)] + [(b >> p) & 1 for p in range(M)]))
    Hb = _brute_hamiltonian(h, g, dets, M)
    Hs = fci.hamiltonian(h, g, 0.0, np.array(s, dtype=np.uint64), np.array(s, dtype=np.uint64)).toarray()
    assert np.max(np.abs(Hb - Hs)) < 1e-12
    assert np.max(np.abs(Hs - Hs.T)) < 1e-12


def test_two_site_hubbard_closed_form():
    gold = _golden("two_site_hubbard.txt")
    h, g = W.hubbard_site(2, gold["t"], gold["U"])
    e = fci.casci(h, g, 0.0, [0], [0, 1])
    assert abs(e - gold["E"]) < 1e-13
    # the same in the bonding/antibonding (MO) basis
    hm, gm = W.hubbard_mo(2, gold["t"], gold["U"])
    assert abs(fci.casci(hm, gm, 0.0, [0], [0, 1]) - gold["E"]) < 1e-13
    # frozen bonding orbital, no active space: the reference-determinant energy
    assert abs(fci.casci(hm, gm, 0.0, [0], []) - gold["E_HF"]) < 1e-13


def test_orbital_rotation_invariance_hubbard8():
    p = W.problem("hubbard8")
    hs, gs = W.hubbard_site(8, 1.0, 2.0)
    e_site = fci.casci(hs, gs, 0.0, p.occ, range(8))
    e_mo = fci.casci(p.h1, p.eri, 0.0, p.occ, range(8))
    assert abs(e_site - e_mo) < 1e-10


def test_dense_and_lanczos_agree():
    p = W.problem("hubbard8")
    a, b = fci.casci_space(p.occ, range(8))
    H = fci.hamiltonian(p.h1, p.eri, 0.0, a, b)
    old = fci.DENSE_MAX
    try:
        fci.DENSE_MAX = 10 ** 9
        e_dense = fci.lowest(H)
        fci.DENSE_MAX = 10
        e_lanczos = fci.lowest(H)
    finally:
        fci.DENSE_MAX = old
    assert abs(e_dense - e_lanczos) < 1e-11


def test_diagonal_matches_matrix():
    h, g = _random_integrals(5, 7)
    a, b = fci.casci_space([0, 1], range(5))
    H = fci.hamiltonian(h, g, 0.25, a, b).toarray()
    assert np.max(np.abs(np.diag(H) - fci.diagonal(h, g, 0.25, a, b))) < 1e-13


def test_sigma_rows_matches_matrix():
    h, g = _random_integrals(6, 11)
    a, b = fci.casci_space([0, 1, 2], range(6))
    H = fci.hamiltonian(h, g, -0.5, a, b)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(H.shape[0])
    rows = rng.choice(H.shape[0], 37, replace=False)
    assert np.max(np.abs(fci.sigma_rows(h, g, -0.5, a, b, c, rows) - (H @ c)[rows])) < 1e-12


def test_frozen_core_equals_explicit_occupation():
    """A frozen doubly occupied orbital is literally present in every determinant:
    the CASCI energy with orbital 0 frozen equals the lowest eigenvalue of the
    whole-space H restricted by hand to determinants with orbital 0 doubly
    occupied and orbital 5 empty."""
    h, g = _random_integrals(6, 3)
    occ = [0, 1, 2]
    active = [1, 2, 3, 4]
    e = fci.casci(h, g, 0.0, occ, active)
    a, b = fci.casci_space(occ, range(6))
    H = fci.hamiltonian(h, g, 0.0, a, b).toarray()
    keep = [ia * len(b) + ib for ia, ma in enumerate(a) for ib, mb in enumerate(b)
            if (int(ma) & 1) and (int(mb) & 1) and not (int(ma) >> 5 & 1) and not (int(mb) >> 5 & 1)]
    w = np.linalg.eigvalsh(H[np.ix_(keep, keep)])
    assert abs(w[0] - e) < 1e-12


def test_variational_monotonicity():
    """Adding an orbital to the active set enlarges the determinant space, so
    the CASCI energy cannot rise."""
    p = W.problem("hubbard8")
    base = [2, 5]
    e0 = fci.casci(p.h1, p.eri, 0.0, p.occ, base)
    for q in range(8):
        if q not in base:
            assert fci.casci(p.h1, p.eri, 0.0, p.occ, sorted(base + [q])) <= e0 + 1e-12


def test_hubbard_integrals():
    h, g = W.hubbard_mo(8, 1.0, 2.0)
    c = W.hubbard_orbitals(8)
    assert np.max(np.abs(c.T @ c - np.eye(8))) < 1e-14
    eps = -2.0 * np.cos(np.pi * np.arange(1, 9) / 9)
    assert np.max(np.abs(h - np.diag(eps))) < 1e-14
    k = np.arange(8)
    parity = (k[:, None, None, None] + k[None, :, None, None] + k[None, None, :, None] + k[None, None, None, :]) % 2
    assert np.max(np.abs(g[parity == 1])) < 1e-14
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.max(np.abs(g - g.transpose(perm))) < 1e-14


def test_synthetic_integrals_symmetry():
    h, g = W.synthetic(10, 0)
    assert np.all(np.diff(np.diag(h)) >= 0)
    assert np.max(np.abs(h - h.T)) == 0.0
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.max(np.abs(g - g.transpose(perm))) < 1e-15
    # positive semidefinite as a pair matrix (sum of outer products)
    w = np.linalg.eigvalsh(g.reshape(100, 100))
    assert w.min() > -1e-12


def test_particle_hole_symmetry_hubbard8():
    """At half filling on a bipartite chain the particle-hole map k -> N+1-k
    sends the CASCI of A (occupied set O) to the CASCI of the mirrored set with
    the same energy."""
    p = W.problem("hubbard8")
    mirror = lambda s: sorted(7 - q for q in s)
    for act in ([0, 4], [1, 2, 6], [0, 3, 4, 7], [2, 3, 5]):
        e1 = fci.casci(p.h1, p.eri, 0.0, p.occ, act)
        e2 = fci.casci(p.h1, p.eri, 0.0, p.occ, mirror(act))
        assert abs(e1 - e2) < 1e-11


def test_paper_determinant_counts():
    """String counts reproduce the determinant counts printed in the paper."""
    with open(os.path.join(GOLDEN, "paper_determinant_counts.txt")) as fh:
        rows = [l.split("#")[0].split('"')[0].split() for l in fh]
    rows = [r for r in rows if r]
    n_checked = 0
    for r in rows:
        if len(r) == 4:
            printed, n, k, tol = float(r[0]), int(r[1]), int(r[2]), float(r[3])
            ndet = len(ostr.strings(n, k)) ** 2 if n <= 14 else math.comb(n, k) ** 2
            assert abs(ndet - printed) / printed < tol
            n_checked += 1
        elif len(r) == 3:
            bound, n, k = float(r[0]), int(r[1]), int(r[2])
            assert math.log10(math.comb(n, k) ** 2) > bound
            n_checked += 1
    assert n_checked == 4


def test_string_tables_small():
    for n, k in [(4, 2), (5, 2), (6, 3)]:
        s = ostr.strings(n, k)
        assert len(s) == math.comb(n, k)
        assert all(bin(m).count("1") == k for m in s)
        assert s == sorted(s)
        t = ostr.link_table(n, k)
        assert all(len(row) == k * (n - k + 1) for row in t)


def test_link_tables_satisfy_commutator():
    """E_pq built from the link tables obey [E_pq, E_rs] = d_qr E_ps - d_ps E_rq."""
    n, k = 5, 2
    t = ostr.link_table(n, k)
    N = len(t)
    E = np.zeros((n, n, N, N))
    for I, row in enumerate(t):
        for p, q, J, s in row:
            E[p, q, J, I] += s
    for p, q, r, s in itertools.product(range(n), repeat=4):
        lhs = E[p, q] @ E[r, s] - E[r, s] @ E[p, q]
        rhs = (q == r) * E[p, s] - (p == s) * E[r, q]
        assert np.max(np.abs(lhs - rhs)) == 0.0
