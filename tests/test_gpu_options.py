"""Solver options of the HIP path (needs an MI355X).  Options change how the
Davidson iteration gets to the eigenpair, never the eigenpair itself:

* the Olsen correction (precond = 1) and the diagonal/P-space correction
  (precond = 0) give the same energies to the convergence tolerance;
* replaying captured graphs (use_graph = 1) and launching every kernel
  (use_graph = 0) run the same kernels in the same order: bitwise equal;
* more guess vectors or a smaller subspace change only the iteration count
  (max_space 3, the smallest, restarts every iteration onto the Ritz vector
  and the previous one);
* forced tile widths give bitwise the autotuned results (the contraction
  order over pairs does not depend on the tiling).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-9


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _forward(p, **opts):
    from paper_1910_03527_amd import Context
    c = Context(0, conv_tol=TOL, **opts)
    try:
        r = c.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order,
                          p.e_const, want_increments=True)
        r["stats"] = dict(c.last_stats)
    finally:
        c.close()
    return r


@pytest.fixture(scope="module")
def hub12():
    p = W.problem("hubbard12")
    _log("options: hubbard12 reference run")
    return p, _forward(p)


@pytest.mark.parametrize("opts", [{"precond": 1}, {"nguess": 3, "max_space": 6},
                                  {"max_space": 3}, {"max_space": 4}, {"max_space": 16},
                                  {"pspace": 0}])
def test_options_reach_the_same_energies(hub12, opts):
    p, ref = hub12
    _log("options", opts)
    got = _forward(p, **opts)
    assert got["stats"]["first_failed"] == -1
    # per-CASCI energy errors are ~|r|^2 / gap; increments and order sums
    # combine a few thousand of them with binomial weights
    assert np.max(np.abs(np.array(got["increments"]) - np.array(ref["increments"]))) < 1e-10
    assert max(abs(a - b) for a, b in zip(got["e_order"], ref["e_order"])) < 1e-9
    assert abs(got["e_total"] - ref["e_total"]) < 1e-9


def test_graph_replay_is_bitwise_plain_launches(hub12):
    p, ref = hub12
    got = _forward(p, use_graph=0)
    assert got["increments"] == ref["increments"] and got["e_order"] == ref["e_order"]
    assert ref["stats"]["graph_launches"] > 0 and got["stats"]["graph_launches"] == 0


@pytest.mark.parametrize("tile", [32, 64, 128])
def test_forced_tiles_bitwise(hub12, tile):
    p, ref = hub12
    got = _forward(p, tile=tile)
    assert got["increments"] == ref["increments"], tile


@pytest.mark.parametrize("tol", [TOL, 1e-7])
def test_olsen_casci_batch(tol):
    """Larger CASCIs (synthetic CAS(10,10), 63,504 determinants) through the
    Olsen correction and through the P-space correction.  Both start from the
    P-space guess: from unit vectors alone the Olsen iteration settled on an
    excited state of the second problem (0.029 E_h up) at 1e-7 and 1e-8."""
    from paper_1910_03527_amd import Context
    probs = [W.synthetic(10, s) for s in (3, 4)]
    es = []
    for opts in ({"precond": 0}, {"precond": 1}):
        c = Context(0, conv_tol=tol, **opts)
        try:
            es.append(c.casci([_dev(h) for h, _ in probs], [_dev(g) for _, g in probs], 5, 5))
            assert c.last_stats["first_failed"] == -1
            # below residual 1e-7 the P-space path switches to the Olsen
            # correction (it took 50 iterations to 1e-9 without the switch)
            assert c.last_stats["max_iters"] <= 35, (opts, c.last_stats["max_iters"])
        finally:
            c.close()
    assert max(abs(a - b) for a, b in zip(*es)) < 1e-10


def test_torch_allocator_workspaces():
    """Workspaces from torch's caching allocator (mbefci_set_allocator): the
    same energies bitwise, the memory counted by torch while the context holds
    it and handed back on close and on switching back to hipMalloc."""
    from paper_1910_03527_amd import Context, MbefciError
    p = W.problem("hubbard12")
    h, g = _dev(p.h1), _dev(p.eri)
    ref = Context(0, conv_tol=TOL)
    r0 = ref.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    c = Context(0, conv_tol=TOL)
    try:
        c.use_torch_allocator()
        r1 = c.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
        held = torch.cuda.memory_allocated() - base
        assert held > 1 << 20, held
        assert r1["increments"] == r0["increments"] and r1["e_order"] == r0["e_order"]
        dh, dg = c.mbe_backward([1.0] * (1 + p.max_order))
        assert torch.isfinite(dh).all() and torch.isfinite(dg).all()
        del dh, dg
        c.use_torch_allocator(False)  # arenas go back to torch, then hipMalloc
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - base < held
        with pytest.raises(MbefciError):
            c.mbe_backward([1.0] * (1 + p.max_order))  # the plan was dropped
        c.use_torch_allocator()
        r2 = c.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
        assert r2["increments"] == r0["increments"]
    finally:
        c.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base <= 0


def test_tolerance_change_reaches_the_cached_plan():
    """A forward at a loose tolerance, then set_opts(conv_tol) and the same
    forward again on the cached plan: it must converge to the new tolerance
    (the captured iteration graph holds the old one and is captured again)."""
    from paper_1910_03527_amd import Context
    p = W.problem("hubbard12")
    h, g = _dev(p.h1), _dev(p.eri)
    c = Context(0, conv_tol=1e-10)
    try:
        ref = c.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
    finally:
        c.close()
    c = Context(0, conv_tol=1e-3)
    try:
        loose = c.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
        it_loose = c.last_stats["max_iters"]
        c.set_opts(conv_tol=1e-10)
        again = c.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, want_increments=True)
        it_again = c.last_stats["max_iters"]
    finally:
        c.close()
    assert it_again > it_loose
    err_loose = abs(loose["e_total"] - ref["e_total"])
    err_again = abs(again["e_total"] - ref["e_total"])
    assert err_again < 1e-10 and err_again < err_loose, (err_loose, err_again)
