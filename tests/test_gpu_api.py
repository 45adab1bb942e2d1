"""The one-CASCI call ``casci`` of the Python binding (needs an MI355X).

* Two-site Hubbard in the site basis (t = 1, U = 2): the energy, the
  one-electron energy and the RDM traces against their closed forms,
  E = (U - sqrt(U^2 + 16 t^2)) / 2 and E_1e = -8 t^2 / sqrt(U^2 + 16 t^2).
* A synthetic CAS(6e,6o) with a core energy: the energy against the oracle's
  Slater-Condon FCI and the batched call, and the RDMs reproducing it.
* ``mbefci_casci`` (one CASCI with its CI vector and RDMs, unequal spins):
  energy, eigenvector (up to sign, via the oracle's eigenvector) and RDMs
  against the oracle; the same CASCI through ``mbefci_casci_batch`` gives
  bitwise the same energy.
* The host integer layer (``mbefci_strings``, ``mbefci_link_table``, no
  context) equals the tables the device kernels build, bit for bit.
* The peak probes return values below the published peaks and within a
  factor of a few of them.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fci
from oracle import rdm as ordm

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


def test_single_casci_with_vector_and_rdms():
    from paper_1910_03527_amd import Context
    n, na, nb = 7, 4, 3
    h, g = W.synthetic(n, 77)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    H = fci.hamiltonian(h, g, 0.25, a, b)
    e_ref, v = fci.lowest(H, want_vec=True)
    v = v / np.linalg.norm(v)
    gam, Gam = ordm.rdm12(a, b, v, n)
    c = Context(0, conv_tol=1e-10)
    try:
        r = c.casci_one(_dev(h), _dev(g), na, nb, 0.25, want_ci=True, want_rdm=True)
        eb = c.casci([_dev(h)], [_dev(g)], na, nb, e_core=[0.25])[0]
    finally:
        c.close()
    assert abs(r["e"] - e_ref) < 1e-9
    assert r["e"] == eb
    ci = r["ci"].cpu().numpy()
    assert abs(np.linalg.norm(ci) - 1.0) < 1e-12
    assert abs(abs(float(ci @ v)) - 1.0) < 1e-9
    assert np.max(np.abs(r["rdm1"].cpu().numpy() - 0.5 * (gam + gam.T))) < 1e-8
    assert np.max(np.abs(r["rdm2"].cpu().numpy() - ordm.sym8(Gam))) < 1e-8


@pytest.mark.parametrize("n,k", [(6, 3), (10, 4), (14, 7)])
def test_host_tables_equal_device_tables(n, k):
    from paper_1910_03527_amd import Context, link_table, strings
    c = Context(0)
    try:
        ds = c.strings(n, k).cpu().numpy().astype(np.uint64)
        dl = c.link_table(n, k).cpu().numpy()
    finally:
        c.close()
    assert np.array_equal(strings(n, k), ds)
    assert np.array_equal(link_table(n, k), dl)


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
