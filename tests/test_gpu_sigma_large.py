"""sigma = H c of the largest compiled kernel shapes, every element against the
matrix-free Slater-Condon oracle (``oracle/direct.py``), needs an MI355X.

The contraction kernel is compiled per active size n; n = 11..14 are reached
by CASCIs of 11-14 orbitals (CAS(12,12) is the size of the paper's benzene
final-order CASCI, CAS(14,14) of its largest Hubbard CASCI).  Each shape is
run with every tile width the kernels have for it (32, 64, and 128 up to 12
orbitals); the whole sigma vector of a seeded random c must agree with the
oracle's to 1e-11 relative to max |sigma|.  The oracle forms each row from the
determinants within two electrons of it, so the comparison covers every
element, not a sample.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, fci

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THREADS = min(16, os.cpu_count() or 1)


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


SHAPES = [(11, 5, 6, (32, 64, 128)), (11, 2, 3, (32, 64, 128)), (12, 6, 6, (32, 64, 128)),
          (12, 3, 4, (32, 64, 128)), (13, 6, 7, (32, 64)), (13, 4, 4, (32, 64)),
          (14, 7, 7, (32, 64))]


@pytest.mark.parametrize("n,na,nb,tiles", SHAPES)
def test_sigma_every_element_matches_oracle(n, na, nb, tiles):
    from paper_1910_03527_amd import Context
    _log("sigma full vector", n, na, nb, tiles)
    if n == 14:
        p = W.problem("cas14", 0)
        h, g = p.h1, p.eri
    else:
        h, g = W.synthetic(n, 600 + 10 * n + na)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    rng = np.random.default_rng(n * 100 + na + nb)
    c = rng.standard_normal(len(a) * len(b))
    c /= np.linalg.norm(c)
    H = direct.DirectHamiltonian(h, g, -0.25, a, b, threads=THREADS)
    try:
        exp = H.matvec(c)
    finally:
        H.close()
    scale = max(1.0, float(np.max(np.abs(exp))))
    hd, gd, cd = _dev(h), _dev(g), _dev(c)
    for tile in tiles:
        ctx = Context(0, tile=tile)
        try:
            got = ctx.sigma(hd, gd, na, nb, cd, -0.25).cpu().numpy()
        finally:
            ctx.close()
        err = float(np.max(np.abs(got - exp)))
        _log("  tile", tile, "ndet", len(c), "max |diff|", err)
        assert err <= 1e-11 * scale, (tile, err)
