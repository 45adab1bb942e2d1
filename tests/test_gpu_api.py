"""The one-CASCI call ``casci`` of the Python binding (needs an MI355X).

* Two-site Hubbard in the site basis (t = 1, U = 2): the energy, the
  one-electron energy and the RDM traces against their closed forms,
  E = (U - sqrt(U^2 + 16 t^2)) / 2 and E_1e = -8 t^2 / sqrt(U^2 + 16 t^2).
* A synthetic CAS(6e,6o) with a core energy: the energy against the oracle's
  Slater-Condon FCI and the batched call, and the RDMs reproducing it.
* The peak probes return values below the published peaks and within a
  factor of a few of them.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fci

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def test_casci_two_site_closed_forms():
    from paper_1910_03527_amd import casci
    t, U = 1.0, 2.0
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0] = g[1, 1, 1, 1] = U
    root = math.sqrt(U * U + 16 * t * t)
    e = casci(_dev(h), _dev(g), 1, 1, conv_tol=1e-10)
    assert abs(e - (U - root) / 2) < 1e-12
    e2, g1, g2 = casci(_dev(h), _dev(g), 1, 1, want_rdm=True, conv_tol=1e-10)
    assert e2 == e
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    assert abs(np.trace(g1) - 2.0) < 1e-12
    assert abs(np.einsum("ppqq->", g2) - 2.0) < 1e-12  # N_e (N_e - 1)
    e1 = float((h * g1).sum())
    assert abs(e1 + 8 * t * t / root) < 1e-10
    assert abs(e1 + 0.5 * float((g * g2).sum()) - e) < 1e-10


def test_casci_synthetic_against_oracle_and_batch():
    from paper_1910_03527_amd import Context, casci
    h, g = W.synthetic(6, 5)
    e_core = 0.375
    ref = fci.casci(h, g, e_core, [0, 1, 2], list(range(6)))
    e, g1, g2 = casci(_dev(h), _dev(g), 3, 3, e_core=e_core, want_rdm=True, conv_tol=1e-10)
    assert abs(e - ref) < 1e-9
    c = Context(0, conv_tol=1e-10)
    try:
        eb = c.casci([_dev(h)], [_dev(g)], 3, 3, e_core=[e_core])[0]
    finally:
        c.close()
    assert eb == e
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    assert abs(np.trace(g1) - 6.0) < 1e-10
    assert abs((h * g1).sum() + 0.5 * (g * g2).sum() + e_core - e) < 1e-9


def test_probe_peaks_plausible():
    from paper_1910_03527_amd import Context
    c = Context(0)
    try:
        pk = c.probe_peaks()
    finally:
        c.close()
    # published: 78.6 TFLOP/s FP64 matrix, 8 TB/s HBM
    assert 20.0 < pk["fp64_mfma_tflops"] < 80.0, pk
    assert 1000.0 < pk["copy_gbps"] < 8200.0, pk
