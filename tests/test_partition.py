"""The Type-1/2/3 partitions of the paper (the discussion before Eq. 3) as
named presets (``mbefci_partition``, host only), and, on the GPU, the
expansion in each partition: full order reaches the whole-space FCI (the
Moebius identity holds for any partition), and a truncated order matches the
oracle's expansion in the same partition."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe
from paper_1910_03527_amd import TYPE1, TYPE2, TYPE3, MbefciError, partition


def test_presets():
    occ = [0, 1, 2, 5]
    assert partition(TYPE1, 8, occ) == ([3, 4, 6, 7], [0, 1, 2, 5])
    assert partition(TYPE2, 8, occ) == ([0, 1, 2, 5], [3, 4, 6, 7])
    assert partition(TYPE3, 8, occ) == ([], list(range(8)))
    with pytest.raises(MbefciError):
        partition(4, 8, occ)
    with pytest.raises(MbefciError):
        partition(TYPE1, 8, [0, 0])


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.gpu
@pytest.mark.parametrize("kind", [TYPE1, TYPE2, TYPE3])
def test_partition_expansions(kind):
    print("partition", kind, flush=True)
    from paper_1910_03527_amd import Context
    h1, g = W.synthetic(8, 77)
    occ = [0, 1, 2, 3]
    ref, exp = partition(kind, 8, occ)
    exact = fci.casci(h1, g, 0.0, occ, range(8))
    c = Context(0, conv_tol=1e-8)
    try:
        full = c.mbe_forward(_dev(h1), _dev(g), occ, ref, exp, len(exp))
        assert abs(full["e_total"] - exact) < 1e-9
        k = 2
        got = c.mbe_forward(_dev(h1), _dev(g), occ, ref, exp, k, want_increments=True)
    finally:
        c.close()
    p = W.Problem("s8", h1, g, 0.0, occ, ref, exp, k)
    r = mbe.mbe(p, workers=min(16, os.cpu_count() or 1))
    assert abs(got["e_ref"] - r["e_ref"]) < 1e-9
    assert np.max(np.abs(np.array(got["increments"]) - np.array(r["inc"]))) < 1e-9
