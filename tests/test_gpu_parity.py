"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Integer work (strings, link tables) must match bit for bit; FP64 results to
the stated tolerances (energies 1e-9 E_h; sigma to 1e-11 relative to the
largest |H_IJ| times |c|_1 -- round-off of sums of a few hundred products).
"""
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe, strings as ostr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_03527_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


# ---------------------------------------------------------------- integers
STRING_SHAPES = [(1, 0), (1, 1), (4, 2), (5, 2), (6, 3), (7, 4), (8, 4), (10, 5), (14, 7), (16, 8)]


@pytest.mark.parametrize("n,k", STRING_SHAPES)
def test_strings_bit_exact(ctx, n, k):
    _log("strings", n, k)
    got = ctx.strings(n, k).cpu().numpy().astype(np.uint64)
    exp = np.array(ostr.strings(n, k), dtype=np.uint64)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n,k", [(2, 1), (4, 2), (5, 3), (6, 3), (8, 4), (10, 5), (14, 7)])
def test_link_tables_bit_exact(ctx, n, k):
    _log("links", n, k)
    got = ctx.link_table(n, k).cpu().numpy()
    exp = np.array(ostr.link_table(n, k), dtype=np.int32)
    assert got.shape == exp.shape
    assert np.array_equal(got, exp)


# ------------------------------------------------------------ one CASCI
def _space(n, na, nb):
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    return a, b


SIGMA_SHAPES = [(2, 1, 1), (3, 1, 2), (4, 2, 2), (5, 2, 3), (6, 3, 3), (7, 3, 4), (8, 4, 4),
                (9, 4, 4), (9, 3, 5), (10, 5, 5)]


@pytest.mark.parametrize("n,na,nb", SIGMA_SHAPES)
def test_hdiag_matches_oracle(ctx, n, na, nb):
    _log("hdiag", n, na, nb)
    h, g = W.synthetic(n, 100 + n)
    a, b = _space(n, na, nb)
    exp = fci.diagonal(h, g, 0.37, a, b)
    got = ctx.hdiag(_dev(h), _dev(g), na, nb, 0.37).cpu().numpy()
    assert np.max(np.abs(got - exp)) < 1e-12 * max(1.0, np.max(np.abs(exp)))


@pytest.mark.parametrize("n,na,nb", SIGMA_SHAPES)
def test_sigma_matches_oracle(ctx, n, na, nb):
    _log("sigma", n, na, nb)
    h, g = W.synthetic(n, 200 + n)
    a, b = _space(n, na, nb)
    rng = np.random.default_rng(n * 100 + na)
    c = rng.standard_normal(len(a) * len(b))
    if len(a) * len(b) <= 20000:
        H = fci.hamiltonian(h, g, -0.25, a, b)
        exp = H @ c
        hmax = np.max(np.abs(H.data))
        rows = np.arange(len(c))
    else:
        rows = np.sort(rng.choice(len(c), 400, replace=False))
        exp = fci.sigma_rows(h, g, -0.25, a, b, c, rows)
        hmax = np.max(np.abs(fci.diagonal(h, g, -0.25, a, b)))
    got = ctx.sigma(_dev(h), _dev(g), na, nb, _dev(c), -0.25).cpu().numpy()[rows]
    err = np.max(np.abs(got - exp))
    assert err <= 1e-11 * max(1.0, np.max(np.abs(exp))), (err, hmax)


def test_sigma_large_cas_sampled_rows(ctx):
    """CAS(14e,14o): 11,778,624 determinants; 256 rows against Slater-Condon."""
    _log("sigma cas14")
    p = W.problem("cas14", 0)
    a, b = _space(14, 7, 7)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(len(a) * len(b))
    c /= np.linalg.norm(c)
    rows = np.sort(rng.choice(len(c), 256, replace=False))
    exp = fci.sigma_rows(p.h1, p.eri, 0.0, a, b, c, rows)
    got = ctx.sigma(_dev(p.h1), _dev(p.eri), 7, 7, _dev(c)).cpu().numpy()[rows]
    assert np.max(np.abs(got - exp)) < 1e-12


CASCI_SHAPES = [(2, 1, 1), (4, 2, 2), (5, 2, 3), (6, 3, 3), (7, 3, 4), (8, 4, 4), (9, 4, 4)]


@pytest.mark.parametrize("n,na,nb", CASCI_SHAPES)
def test_casci_energy_matches_oracle(ctx, n, na, nb):
    _log("casci", n, na, nb)
    h, g = W.synthetic(n, 300 + n)
    a, b = _space(n, na, nb)
    exp = fci.lowest(fci.hamiltonian(h, g, 0.5, a, b))
    got = ctx.casci([_dev(h)], [_dev(g)], na, nb, [0.5])[0]
    assert abs(got - exp) < 1e-9, (got, exp)


def test_casci_hubbard8_whole_space(ctx):
    _log("casci hubbard8")
    p = W.problem("hubbard8")
    exp = fci.casci(p.h1, p.eri, 0.0, p.occ, range(8))
    got = ctx.casci([_dev(p.h1)], [_dev(p.eri)], 4, 4)[0]
    assert abs(got - exp) < 1e-9


def test_casci_batch_matches_single(ctx):
    _log("casci batch")
    hs, gs, exp = [], [], []
    for s in range(3):
        h, g = W.synthetic(7, 400 + s)
        hs.append(_dev(h))
        gs.append(_dev(g))
        exp.append(ctx.casci([hs[-1]], [gs[-1]], 3, 3)[0])
    got = ctx.casci(hs, gs, 3, 3)
    assert max(abs(x - y) for x, y in zip(got, exp)) < 1e-10


# ---------------------------------------------------------------- MBE
_ORACLE = {}


def _oracle_mbe(name):
    if name not in _ORACLE:
        p = W.problem(name)
        _ORACLE[name] = (p, mbe.mbe(p, workers=min(16, os.cpu_count() or 1)))
    return _ORACLE[name]


def _gpu_mbe(ctx, p, **kw):
    return ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order, p.e_const,
                           want_increments=True, **kw)


@pytest.mark.parametrize("name", ["hubbard8", "hubbard12"])
def test_mbe_matches_oracle(ctx, name):
    _log("mbe", name)
    p, r = _oracle_mbe(name)
    got = _gpu_mbe(ctx, p)
    assert abs(got["e_ref"] - r["e_ref"]) < 1e-9
    assert np.max(np.abs(np.array(got["increments"]) - np.array(r["inc"]))) < 1e-9
    assert np.max(np.abs(np.array(got["e_order"]) - np.array(r["e_order"]))) < 1e-9
    assert abs(got["e_total"] - r["e_total"]) < 1e-9


def test_mbe_full_order_equals_fci(ctx):
    _log("mbe full order")
    p = W.problem("hubbard8")
    got = _gpu_mbe(ctx, p)
    assert abs(got["e_total"] - fci.casci(p.h1, p.eri, 0.0, p.occ, range(8))) < 1e-9


def test_mbe_per_launch_equals_batched(ctx):
    _log("mbe per-launch")
    from paper_1910_03527_amd import PER_LAUNCH, BATCHED
    p = W.problem("hubbard8")
    b = _gpu_mbe(ctx, p)
    ctx.set_opts(mode=PER_LAUNCH)
    try:
        s = _gpu_mbe(ctx, p)
    finally:
        ctx.set_opts(mode=BATCHED)
    assert np.max(np.abs(np.array(b["increments"]) - np.array(s["increments"]))) < 1e-10


def test_mbe_deterministic(ctx):
    _log("mbe determinism")
    p = W.problem("hubbard12")
    a = _gpu_mbe(ctx, p)
    b = _gpu_mbe(ctx, p)
    assert a["increments"] == b["increments"] and a["e_order"] == b["e_order"]


def test_large_casci_batched_equals_per_launch():
    """CASCIs above 16,384 determinants select their P-space in chunks; in
    per-launch mode each CASCI is a view of its own.  Both modes give
    bitwise the same energies (same kernels, same work per CASCI), and both
    CAS(12,12) energies equal the oracle's matrix-free Lanczos values of
    tests/golden/casci_large.txt to 1e-9 E_h."""
    from golden_io import read_large_goldens
    from paper_1910_03527_amd import Context, PER_LAUNCH
    probs = [W.synthetic(12, s) for s in (21, 22)]   # CAS(12e,12o): 853,776 determinants
    hs = [_dev(h) for h, _ in probs]
    gs = [_dev(g) for _, g in probs]
    _log("large casci batched vs per-launch")
    a = Context(0)
    try:
        ea = a.casci(hs, gs, 6, 6)
    finally:
        a.close()
    b = Context(0, mode=PER_LAUNCH)
    try:
        eb = b.casci(hs, gs, 6, 6)
    finally:
        b.close()
    assert max(abs(x - y) for x, y in zip(ea, eb)) < 1e-10
    golden = read_large_goldens()
    for e, key in zip(ea, ("cas12_21", "cas12_22")):
        assert abs(e - golden[key]) < 1e-9, (key, e, golden[key])
