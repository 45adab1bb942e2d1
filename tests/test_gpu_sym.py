"""Point-group blocked CASCIs on the HIP path (needs an MI355X), against the
oracle's CASCI in one irrep (``oracle/sym.py``), on synthetic Hamiltonians
whose integrals respect D2h (``workloads.synthetic_sym``).  The paper solves
its Cr2 CASCIs with D2h symmetry (Fig. 3 discussion).

* sigma = H c on the determinants of one irrep, every element against the
  oracle's sector Hamiltonian, for several shapes and target irreps (the CI
  vector's blocked layout is the one include/mbefci.h documents: strings
  sorted by (irrep, bitmask), blocks over alpha irreps).
* CASCI energies in every irrep against the oracle (1e-9 E_h); eigenvectors
  against the oracle's up to sign.
* The screened expansion with orbital irreps (every CASCI in the totally
  symmetric irrep) against the oracle's: tuple sets exact, increments, order
  sums and totals to 1e-9 E_h; with T_init = 0 it is the full expansion.
* At CAS(14,14) size: the blocked sigma of a vector of the totally symmetric
  irrep equals the plain (unblocked, separately pinned) sigma of that vector
  embedded in the full product space, restricted back.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, fci, screen, sym

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def blocked_positions(a, b, orbsym, G):
    """For the product-space sector indices of irrep G (oracle order), their
    positions in the blocked layout."""
    ia_irr = np.array([sym.string_irrep(m, orbsym) for m in a])
    ib_irr = np.array([sym.string_irrep(m, orbsym) for m in b])

    def ranks(irr):
        r = np.zeros(len(irr), dtype=np.int64)
        cnt = np.zeros(8, dtype=np.int64)
        for i, x in enumerate(irr):  # ascending bitmask within an irrep
            r[i] = cnt[x]
            cnt[x] += 1
        return r, cnt

    ra, ca = ranks(ia_irr)
    rb, cb = ranks(ib_irr)
    blk = np.zeros(9, dtype=np.int64)
    for x in range(8):
        blk[x + 1] = blk[x] + ca[x] * cb[x ^ G]
    idx = sym.sector(a, b, orbsym, G)
    ia, ib = idx // len(b), idx % len(b)
    pos = blk[ia_irr[ia]] + ra[ia] * cb[ia_irr[ia] ^ G] + rb[ib]
    assert np.array_equal(np.sort(pos), np.arange(len(idx)))
    return idx, pos


SIGMA_CASES = [
    (6, 3, 3, [0, 1, 2, 3, 0, 1], 0, 31),
    (6, 3, 3, [0, 1, 2, 3, 0, 1], 3, 31),
    (7, 3, 4, [1, 4, 4, 7, 0, 2, 3], 5, 32),
    (8, 4, 4, [0, 5, 3, 6, 0, 1, 7, 2], 0, 33),
    (9, 4, 4, [0, 0, 1, 1, 2, 3, 4, 5, 6], 6, 34),
    (10, 5, 5, [p % 8 for p in range(10)], 0, 35),
    (10, 4, 5, [0] * 10, 0, 36),   # one irrep (C1): every pair in class 0
    (12, 6, 6, [p // 2 % 8 for p in range(12)], 0, 37),
]


@pytest.mark.parametrize("n,na,nb,osym,G,seed", SIGMA_CASES)
def test_blocked_sigma_matches_oracle(n, na, nb, osym, G, seed):
    from paper_1910_03527_amd import Context, sym_ndet
    _log("blocked sigma", n, na, nb, osym, G)
    h, g = W.synthetic_sym(n, seed, osym)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    nd = sym_ndet(n, na, nb, osym, G)
    idx, pos = blocked_positions(a, b, osym, G)
    assert nd == len(idx)
    rng = np.random.default_rng(seed)
    c_or = rng.standard_normal(nd)
    if len(a) * len(b) <= 60000:
        Hs, idx2 = sym.hamiltonian(h, g, 0.3, a, b, osym, G)
        assert np.array_equal(idx, idx2)
        exp_or = Hs @ c_or
    else:
        # larger spaces: the matrix-free Slater-Condon operator on the whole
        # product space, applied to the sector vector embedded with zeros (H
        # couples no two irreps for these integrals), restricted back
        D = direct.DirectHamiltonian(h, g, 0.3, a, b, threads=min(16, os.cpu_count() or 1))
        try:
            full = np.zeros(len(a) * len(b))
            full[idx] = c_or
            out = D.matvec(full)
        finally:
            D.close()
        other = np.ones(len(full), dtype=bool)
        other[idx] = False
        assert np.max(np.abs(out[other])) < 1e-12
        exp_or = out[idx]
    c_bl = np.empty(nd)
    c_bl[pos] = c_or
    ctx = Context(0)
    try:
        got = ctx.sigma_sym(_dev(h), _dev(g), na, nb, osym, G, _dev(c_bl), 0.3).cpu().numpy()
    finally:
        ctx.close()
    err = float(np.max(np.abs(got[pos] - exp_or)))
    _log("  ndet", nd, "max |diff|", err)
    assert err <= 1e-11 * max(1.0, float(np.max(np.abs(exp_or))))


CASCI_CASES = [
    (6, 3, 3, [0, 1, 2, 3, 0, 1], 41),
    (8, 4, 4, [0, 5, 3, 6, 0, 1, 7, 2], 42),
    (8, 3, 4, [1, 1, 2, 0, 0, 4, 5, 2], 43),
]


@pytest.mark.parametrize("n,na,nb,osym,seed", CASCI_CASES)
def test_blocked_casci_every_irrep_matches_oracle(n, na, nb, osym, seed):
    from paper_1910_03527_amd import Context, sym_ndet
    _log("blocked casci", n, na, nb, osym)
    h, g = W.synthetic_sym(n, seed, osym)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    ctx = Context(0, conv_tol=1e-9, max_iter=400)
    try:
        for G in range(8):
            nd = sym_ndet(n, na, nb, osym, G)
            if nd == 0:
                continue
            Hs, idx = sym.hamiltonian(h, g, 0.125, a, b, osym, G)
            e_ref, v = fci.lowest(Hs, want_vec=True)
            e, cis = ctx.casci_sym([_dev(h)], [_dev(g)], na, nb, osym, G, e_core=[0.125],
                                   want_ci=True)
            _, pos = blocked_positions(a, b, osym, G)
            ci = cis[0].cpu().numpy()
            _log("  irrep", G, "ndet", nd, "E", e[0], "oracle", e_ref)
            assert abs(e[0] - e_ref) < 1e-9, G
            assert abs(abs(float(ci[pos] @ v)) / np.linalg.norm(v) - 1.0) < 1e-8, G
    finally:
        ctx.close()


def _sym_problem(k):
    osym = [0, 5, 3, 6, 0, 1, 7, 2, 3]
    h, g = W.synthetic_sym(9, 51, osym)
    return W.Problem("sym9", h, g, 0.0, [0, 1, 2, 3], [], list(range(9)), k, orbsym=osym)


@pytest.mark.parametrize("t_init,m_init,k", [(0.0, 3, 9), (1e-6, 2, 9)])
def test_blocked_screened_expansion_matches_oracle(t_init, m_init, k):
    from paper_1910_03527_amd import Context
    p = _sym_problem(k)
    _log("blocked screened", t_init, k)
    occ = set(p.occ)
    ref = screen.screened_mbe(p, t_init, m_init, 5.0, max_order=k,
                              workers=min(16, os.cpu_count() or 1))
    margin = min((abs(abs(d) - screen.threshold(t, occ, t_init, m_init, 5.0))
                  for lvl in ref["per_order"] for t, d in lvl), default=1.0)
    assert t_init == 0.0 or margin > 1e-8
    ctx = Context(0, conv_tol=1e-8)
    try:
        got = ctx.mbe_screened(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, k, t_init, m_init,
                               5.0, want_tuples=True, orbsym=p.orbsym)
    finally:
        ctx.close()
    assert abs(got["e_ref"] - ref["e_ref"]) < 1e-9
    for n in range(k):
        tu, inc = got["per_order"][n]
        assert [tuple(int(x) for x in row) for row in tu] == [t for t, _ in ref["per_order"][n]]
        if len(inc):
            exp_d = np.array([d for _, d in ref["per_order"][n]])
            assert np.max(np.abs(np.array(inc) - exp_d)) < 1e-9, n + 1
        assert abs(got["e_order"][n] - ref["e_order"][n]) < 1e-9
    assert abs(got["e_total"] - ref["e_total"]) < 1e-9
    if t_init == 0.0 and k == 9:
        exact = sym.casci(p.h1, p.eri, 0.0, p.occ, range(9), p.orbsym, 0)
        assert abs(got["e_total"] - exact) < 1e-9


def test_blocked_sigma_cas14_equals_plain_sigma():
    from paper_1910_03527_amd import Context, sym_ndet
    n = 14
    osym = [p // 2 % 8 for p in range(n)]
    h, g = W.synthetic_sym(n, 61, osym)
    a = fci.string_masks(range(n), 7)
    nd = sym_ndet(n, 7, 7, osym, 0)
    _log("blocked cas14 sigma", nd, "of", len(a) ** 2)
    idx, pos = blocked_positions(a, a, osym, 0)
    rng = np.random.default_rng(9)
    c_bl = rng.standard_normal(nd)
    c_bl /= np.linalg.norm(c_bl)
    c_full = np.zeros(len(a) * len(a))
    c_full[idx] = c_bl[pos]
    ctx = Context(0)
    try:
        hd, gd = _dev(h), _dev(g)
        s_bl = ctx.sigma_sym(hd, gd, 7, 7, osym, 0, _dev(c_bl)).cpu().numpy()
        s_full = ctx.sigma(hd, gd, 7, 7, _dev(c_full)).cpu().numpy()
    finally:
        ctx.close()
    # the plain sigma of a totally symmetric vector stays in that irrep
    other = np.ones(len(c_full), dtype=bool)
    other[idx] = False
    assert np.max(np.abs(s_full[other])) < 1e-13
    err = float(np.max(np.abs(s_bl[pos] - s_full[idx])))
    _log("  max |blocked - plain|", err)
    assert err < 1e-12 * max(1.0, float(np.max(np.abs(s_full))))


def test_blocked_cas14_lowest_irrep_equals_plain_energy():
    """Full size: the lowest of the eight blocked CAS(14,14) energies equals
    the plain solver's lowest eigenvalue of the same D2h-symmetric
    Hamiltonian (the sectors partition the spectrum)."""
    from paper_1910_03527_amd import Context, sym_ndet
    p = W.problem("cas14_d2h", 0)
    osym = p.orbsym
    ctx = Context(0, conv_tol=1e-7)
    try:
        hd, gd = _dev(p.h1), _dev(p.eri)
        e_plain = ctx.casci([hd], [gd], 7, 7)[0]
        eg = []
        for G in range(8):
            if sym_ndet(14, 7, 7, osym, G) == 0:
                continue
            eg.append((ctx.casci_sym([hd], [gd], 7, 7, osym, G)[0], G))
    finally:
        ctx.close()
    _log("  plain", e_plain, "blocked per irrep", eg)
    assert abs(min(eg)[0] - e_plain) < 1e-9
