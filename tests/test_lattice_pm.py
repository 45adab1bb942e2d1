"""Localised-orbital Hubbard lattices (the paper's Type-3 lattice runs): the
Pipek-Mezey input orbitals, the Lieb-Wu reference energy and the oracle's
expansion on that basis.  CPU only.

Pins that do not come from the code under test:
* localisation: orthonormal columns, unchanged occupied and virtual spans
  (the reference determinant is the same), a stationary point of the
  locality sum checked by brute force over rotation angles;
* Lieb-Wu: the U -> 0 limit -4/pi (the free open band's bulk value),
  the strong-coupling limit -4 ln2 / U, and E/N = -0.57373 at U = 4;
* expansion: full order with no screening equals the FCI energy of the
  same lattice in the canonical basis (basis invariance plus the telescoping
  of Eq. 2); at U = 0 the reference determinant is exact, so every CASCI
  equals E_ref and every increment vanishes.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe, screen


def _locality(c):
    return float(np.sum(c ** 4))


@pytest.mark.parametrize("nsite", [8, 10, 22])
def test_pm_orbitals_orthonormal_and_span(nsite):
    h, g, c = W.hubbard_pm(nsite, 1.0, 2.0)
    assert np.allclose(c.T @ c, np.eye(nsite), atol=1e-12)
    c0 = W.hubbard_orbitals(nsite)
    k = nsite // 2
    assert np.allclose(c[:, :k] @ c[:, :k].T, c0[:, :k] @ c0[:, :k].T, atol=1e-12)
    assert np.allclose(c[:, k:] @ c[:, k:].T, c0[:, k:] @ c0[:, k:].T, atol=1e-12)
    # the one-body matrix stays the hopping matrix in a rotated basis
    hs, _ = W.hubbard_site(nsite, 1.0, 2.0)
    assert np.allclose(c @ h @ c.T, hs, atol=1e-12)
    # locality grows from the canonical orbitals
    assert _locality(c[:, :k]) > 2.0 * _locality(c0[:, :k])


def test_pm_stationary_by_brute_force():
    _, _, c = W.hubbard_pm(10, 1.0, 2.0)
    angles = np.linspace(-math.pi / 4, math.pi / 4, 721)
    for block in (c[:, :5], c[:, 5:]):
        base = _locality(block)
        for s, t in itertools.combinations(range(5), 2):
            x, y = block[:, s], block[:, t]
            best = max(np.sum((math.cos(a) * x + math.sin(a) * y) ** 4 +
                              (-math.sin(a) * x + math.cos(a) * y) ** 4) -
                       np.sum(x ** 4 + y ** 4) for a in angles)
            assert best < 1e-10, (s, t, best, base)


def test_pm_orbitals_are_local_and_ordered():
    _, _, c = W.hubbard_pm(22, 1.0, 2.0)
    sites = np.arange(22)
    for blk in (c[:, :11], c[:, 11:]):
        cen = sites @ (blk * blk)
        assert np.all(np.diff(cen) > 0)
        # each orbital keeps most of its weight within two sites of its centroid
        for i in range(11):
            w = blk[:, i] ** 2
            assert w[np.abs(sites - cen[i]) <= 2.0].sum() > 0.85
        big = np.argmax(np.abs(blk), axis=0)
        assert np.all(blk[big, np.arange(11)] > 0)


def test_pm_integrals_symmetric():
    p = W.problem("hubbard10_pm")
    g = p.eri
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.allclose(g, g.transpose(perm), atol=1e-13)
    assert np.allclose(p.h1, p.h1.T)
    assert p.ref == [] and p.exp == list(range(10)) and p.occ == list(range(5))
    assert W.problem("hubbard22_pm").max_order == 14
    assert W.problem("hubbard10_pm_u3").eri[0, 0, 0, 0] > p.eri[0, 0, 0, 0]


def test_lieb_wu_limits():
    assert abs(W.lieb_wu_energy(0.0) + 4.0 / math.pi) < 1e-6
    for u in (40.0, 100.0):
        e = W.lieb_wu_energy(u)
        assert abs(e / (-4.0 * math.log(2.0) / u) - 1.0) < 3.0 / u ** 2 * 10
    assert abs(W.lieb_wu_energy(4.0) + 0.57373) < 5e-5
    es = [W.lieb_wu_energy(u) for u in (0.5, 1.0, 2.0, 3.0)]
    assert all(a < b for a, b in zip(es, es[1:]))


def test_reference_energy_invariant_under_localisation():
    pm = W.problem("hubbard10_pm")
    can = W.problem("hubbard10")
    # hubbard10 (generic name) uses U = 2, the same as hubbard10_pm
    e_pm = fci.casci(pm.h1, pm.eri, 0.0, pm.occ, [])
    e_can = fci.casci(can.h1, can.eri, 0.0, can.occ, [])
    assert abs(e_pm - e_can) < 1e-11


def test_full_order_equals_canonical_fci():
    p = W.problem("hubbard8_pm")
    r = screen.screened_mbe(p, 0.0, 3, 5.0, max_order=8, workers=8)
    can = W.problem("hubbard8")
    e_fci = fci.casci(can.h1, can.eri, 0.0, can.occ, list(range(8)))
    assert abs(r["e_total"] - e_fci) < 1e-9
    # every non-structural tuple is computed: the mixed ones
    n_mixed = sum(math.comb(8, k) - 2 * math.comb(4, k) for k in range(2, 9))
    assert sum(len(lvl) for lvl in r["per_order"]) == n_mixed


def test_free_lattice_increments_vanish():
    h, g, _ = W.hubbard_pm(10, 1.0, 0.0)
    p = W.Problem("free10_pm", h, g, 0.0, list(range(5)), [], list(range(10)), 3)
    r = mbe.mbe(p, max_order=3, workers=8)
    e_free = 2.0 * sum(-2.0 * math.cos(math.pi * k / 11) for k in range(1, 6))
    assert abs(r["e_ref"] - e_free) < 1e-12
    assert max(abs(x) for x in r["e_order"]) < 1e-11
