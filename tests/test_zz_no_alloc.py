"""mbefci_sigma_noalloc (sigma = H c from the library's static scratch array,
no device allocation) against mbefci_sigma on the same inputs, through the
C ABI (needs an MI355X).

* Calls in a row on one GPU, largest first (CAS(10,10) at 5+5 electrons, the
  biggest shape the 32 MiB scratch holds), then smaller and unbalanced
  shapes, then a single-determinant space: each must agree with
  mbefci_sigma element by element to 1e-12 relative to max |sigma| (the
  same kernels run on the same operands, so the values are expected to be
  bitwise equal; the bound leaves room for a different tiling).
* A shape whose tables and G exceed the scratch is rejected on the host
  with ENOMEM and a message naming the size, before any launch.
* The context's own calls are unaffected: mbefci_sigma gives the same result
  before and after the no-allocation calls.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


SHAPES = [(10, 5, 5, 11), (7, 4, 3, 12), (9, 4, 4, 13), (4, 4, 0, 14), (6, 2, 2, 15)]


def test_noalloc_sigma_matches_sigma():
    from paper_1910_03527_amd import Context, num_strings
    ctx = Context(0)
    try:
        first = None
        for n, na, nb, seed in SHAPES:
            _log("sigma_noalloc", n, na, nb, seed)
            h1, g = W.synthetic(n, seed)
            nd = num_strings(n, na) * num_strings(n, nb)
            rng = np.random.default_rng(seed)
            cv = rng.standard_normal(nd)
            cv /= np.linalg.norm(cv)
            h1d, gd, cd = _dev(h1), _dev(g), _dev(cv)
            e_core = 0.25 * seed
            ref = ctx.sigma(h1d, gd, na, nb, cd, e_core).cpu().numpy()
            out = torch.full((nd,), float("nan"), dtype=torch.float64, device="cuda")
            got = ctx.sigma_noalloc(h1d, gd, na, nb, cd, out, e_core)
            torch.cuda.synchronize()
            got = got.cpu().numpy()
            scale = max(1.0, float(np.max(np.abs(ref))))
            err = float(np.max(np.abs(got - ref)))
            _log("  ndet", nd, "max |diff|", err, "bitwise", bool(np.array_equal(got, ref)))
            assert np.all(np.isfinite(got))
            assert err <= 1e-12 * scale
            if first is None:
                first = (h1d, gd, cd, na, nb, e_core, ref)
        # the context's own sigma after the no-allocation calls: unchanged
        h1d, gd, cd, na, nb, e_core, ref = first
        again = ctx.sigma(h1d, gd, na, nb, cd, e_core).cpu().numpy()
        assert np.array_equal(again, ref)
    finally:
        ctx.close()


def test_noalloc_sigma_rejects_oversize_shape():
    from paper_1910_03527_amd import Context, MbefciError, num_strings
    ctx = Context(0)
    try:
        n, na, nb = 11, 5, 5  # G alone is 113 MB
        h1, g = W.synthetic(n, 3)
        nd = num_strings(n, na) * num_strings(n, nb)
        cd = torch.zeros(nd, dtype=torch.float64, device="cuda")
        out = torch.zeros(nd, dtype=torch.float64, device="cuda")
        with pytest.raises(MbefciError) as ei:
            ctx.sigma_noalloc(_dev(h1), _dev(g), na, nb, cd, out)
        assert "ENOMEM" in str(ei.value) and "bytes of scratch" in str(ei.value)
    finally:
        ctx.close()
