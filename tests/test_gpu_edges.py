"""Edge cases of the HIP path (needs an MI355X): empty and degenerate
expansions, single-determinant CASCIs, the largest orbital count (M = 64),
open-shell-only spin sectors, and the error paths of the C ABI."""
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def ctx():
    from paper_1910_03527_amd import Context
    c = Context(0)
    yield c
    c.close()


def _fwd(ctx, p, k=None, **kw):
    return ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp,
                           p.max_order if k is None else k, p.e_const, **kw)


def test_order_zero_is_the_reference_casci(ctx):
    _log("order 0")
    h1, g = W.hubbard_mo(8, 1.0, 2.0)
    p = W.Problem("h8r", h1, g, 0.0, [0, 1, 2, 3], [2, 3, 4, 5], [0, 1, 6, 7], 0)
    r = _fwd(ctx, p)
    e = fci.casci(h1, g, 0.0, p.occ, p.ref)
    assert abs(r["e_ref"] - e) < 1e-9 and r["e_order"] == [] and r["e_total"] == r["e_ref"]
    q = W.Problem("h8e", h1, g, 0.0, [0, 1, 2, 3], [2, 3, 4, 5], [], 0)
    assert abs(_fwd(ctx, q)["e_ref"] - e) < 1e-9


def test_single_determinant_expansion(ctx):
    """Vacuum reference, expansion over occupied MOs only: every CASCI is the
    reference determinant itself, every increment vanishes (Eq. 3)."""
    _log("single-determinant tuples")
    h1, g = W.hubbard_mo(8, 1.0, 2.0)
    p = W.Problem("h8o", h1, g, 0.0, [0, 1, 2, 3], [], [0, 1, 2, 3], 3)
    r = _fwd(ctx, p, want_increments=True)
    st = ctx.last_stats
    assert st["nsingle"] == st["ntuples"]
    assert np.max(np.abs(r["increments"])) < 1e-12
    assert abs(r["e_total"] - fci.casci(h1, g, 0.0, p.occ, [])) < 1e-10


def test_noninteracting_limit(ctx):
    """U = 0: the reference determinant is exact; every increment is zero."""
    _log("U = 0")
    h1, g = W.hubbard_mo(8, 1.0, 0.0)
    p = W.Problem("h8u0", h1, g, 0.0, [0, 1, 2, 3], [], list(range(8)), 4)
    r = _fwd(ctx, p, want_increments=True)
    assert np.max(np.abs(r["increments"])) < 1e-10


def test_largest_orbital_count(ctx):
    """M = 64 (the largest supported): frozen core of 60 orbitals' worth of
    integrals folded into each CASCI, checked against the oracle."""
    _log("M = 64")
    h1, g = W.synthetic(64, 5)
    occ = list(range(10))
    p = W.Problem("s64", h1, g, 0.0, occ, [8, 9, 10, 11], [5, 6, 7, 12, 13, 14], 2)
    r = _fwd(ctx, p, want_increments=True)
    o = mbe.mbe(p, workers=min(16, os.cpu_count() or 1))
    assert abs(r["e_ref"] - o["e_ref"]) < 1e-9
    assert np.max(np.abs(np.array(r["increments"]) - np.array(o["inc"]))) < 1e-9


def test_largest_orbital_count_backward():
    """The backward at M = 64 with orbital 63 in the expansion space (the top
    bit of the 64-bit orbital masks, 2,016 orbital pairs) against the
    oracle's gradient; the gradients are exactly symmetric.  The RDMs are
    first order in the CI vector's error, hence the tight residual."""
    from oracle import rdm as ordm
    from paper_1910_03527_amd import Context
    _log("M = 64 backward")
    h1, g = W.synthetic(64, 5)
    p = W.Problem("s64b", h1, g, 0.0, list(range(10)), [8, 9, 10, 11], [5, 6, 12, 63], 2)
    gvec = [0.7, 1.0, -0.4]
    c = Context(0, conv_tol=1e-10)
    try:
        c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order, p.e_const)
        dh, dg = c.mbe_backward(gvec)
        dh, dg = dh.cpu().numpy(), dg.cpu().numpy()
    finally:
        c.close()
    dh_o, dg_o, _, _ = ordm.mbe_gradient(p, gvec[0], gvec[1:], workers=min(16, os.cpu_count() or 1))
    assert np.max(np.abs(dh - dh_o)) < 1e-8
    assert np.max(np.abs(dg - dg_o)) < 1e-8
    assert np.max(np.abs(dg_o[63])) > 1e-6  # orbital 63 does enter
    assert np.array_equal(dh, dh.T)
    assert np.array_equal(dg, dg.transpose(2, 3, 0, 1))


@pytest.mark.parametrize("n,na,nb", [(4, 2, 0), (5, 0, 3), (6, 1, 4), (7, 7, 2)])
def test_unbalanced_spin_sectors(ctx, n, na, nb):
    _log("casci", n, na, nb)
    h, g = W.synthetic(n, 900 + n)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    exp = fci.lowest(fci.hamiltonian(h, g, 0.1, a, b))
    got = ctx.casci([_dev(h)], [_dev(g)], na, nb, [0.1])[0]
    assert abs(got - exp) < 1e-9


def _bad_problems():
    h1, g = W.hubbard_mo(8, 1.0, 2.0)
    occ = [0, 1, 2, 3]
    hn = h1.copy()
    hn[0, 1] += 1e-6                      # not symmetric
    gn = g.copy()
    gn[1, 2, 3, 4] = np.nan               # not finite
    ga = g.copy()
    ga[0, 1, 2, 3] += 1e-6                # one element without its 8-fold partners
    hi = h1.copy()
    hi[2, 2] = np.inf                     # not finite
    big = list(range(8))
    return [
        ("overlap", (h1, g, occ, [0, 1], [1, 2, 3], 2), "EINVAL"),
        ("range", (h1, g, occ, [], [0, 8], 1), "EINVAL"),
        ("order", (h1, g, occ, [], [0, 1], 3), "EINVAL"),
        ("dup_occ", (h1, g, [0, 0, 1], [], [2, 3], 1), "EINVAL"),
        ("asym_h", (hn, g, occ, [], big, 2), "EINVAL"),
        ("nan_eri", (h1, gn, occ, [], big, 2), "EINVAL"),
        ("asym_eri", (h1, ga, occ, [], big, 2), "EINVAL"),
        ("inf_h", (hi, g, occ, [], big, 2), "EINVAL"),
    ]


@pytest.mark.parametrize("name,args,code", _bad_problems(), ids=[b[0] for b in _bad_problems()])
def test_invalid_problems_are_rejected(ctx, name, args, code):
    from paper_1910_03527_amd import MbefciError
    from paper_1910_03527_amd import _lib
    h1, g, occ, ref, exp, k = args
    with pytest.raises(MbefciError) as ei:
        ctx.mbe_forward(_dev(h1), _dev(g), occ, ref, exp, k)
    assert ei.value.code == getattr(_lib, code)
    # the context stays usable
    p = W.problem("hubbard8")
    assert abs(_fwd(ctx, p, 2)["e_ref"] - fci.casci(p.h1, p.eri, 0.0, p.occ, [])) < 1e-9


def test_active_space_beyond_compiled_kernels(ctx):
    from paper_1910_03527_amd import MbefciError, _lib
    h1, g = W.synthetic(20, 3)
    with pytest.raises(MbefciError) as ei:
        ctx.mbe_forward(_dev(h1), _dev(g), list(range(8)), list(range(12)), list(range(12, 20)), 3)
    assert ei.value.code == _lib.EUNSUPPORTED


def test_backward_needs_forward():
    """Through the C ABI: a backward on a context without a forward is EINVAL."""
    import ctypes
    from paper_1910_03527_amd import Context, _lib
    c = Context(0)
    try:
        g = (ctypes.c_double * 2)(1.0, 1.0)
        dh = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
        dg = torch.zeros((8,) * 4, dtype=torch.float64, device="cuda")
        rc = c._L.mbefci_mbe_backward(c._h, g, ctypes.c_void_p(dh.data_ptr()),
                                      ctypes.c_void_p(dg.data_ptr()), None)
        assert rc == _lib.EINVAL
    finally:
        c.close()


def test_iteration_limit_reports_enotconv():
    """max_iter = 1 forced from the host: the expansion fails with ENOTCONV
    naming the first CASCI that did not converge; the context stays usable."""
    from paper_1910_03527_amd import Context, MbefciError, _lib
    p = W.problem("hubbard12")
    c = Context(0, max_iter=1)
    try:
        with pytest.raises(MbefciError) as ei:
            c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order)
        assert ei.value.code == _lib.ENOTCONV
        assert "did not converge for CASCI" in str(ei.value)
        c.set_opts(max_iter=200)
        r = c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order)
        assert c.last_stats["first_failed"] == -1 and math.isfinite(r["e_total"])
    finally:
        c.close()


def test_workspace_cap_reports_enomem():
    """A workspace cap below what the expansion needs: ENOMEM before any
    launch that needs the memory; lifting the cap makes it run."""
    from paper_1910_03527_amd import Context, MbefciError, _lib
    p = W.problem("hubbard12")
    c = Context(0, max_workspace=1 << 20)
    try:
        with pytest.raises(MbefciError) as ei:
            c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order)
        assert ei.value.code == _lib.ENOMEM
        c.set_opts(max_workspace=0)
        r = c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order)
        assert math.isfinite(r["e_total"])
    finally:
        c.close()
