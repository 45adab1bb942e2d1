"""Pins of the oracle's many-body expansion (Eq. 1-3) and RDM gradients."""
import itertools
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe, rdm

from test_oracle_fci import _golden


@pytest.fixture(scope="module")
def hub8():
    p = W.problem("hubbard8")
    return p, mbe.mbe(p, workers=min(8, os.cpu_count() or 1))


def test_tuple_counts():
    assert len(mbe.tuples(range(8), 8)) == 255
    assert len(mbe.tuples(range(10), 4)) == 385
    assert len(mbe.tuples(range(34), 3)) == 6579
    assert len(mbe.tuples(range(12), 6)) == 2509


def test_full_order_equals_whole_space_fci(hub8):
    """The complete expansion telescopes to the whole-space FCI energy."""
    p, r = hub8
    e_fci = fci.casci(p.h1, p.eri, 0.0, p.occ, range(8))
    assert abs(r["e_total"] - e_fci) < 1e-10


def test_vacuum_reference_zero_increments(hub8):
    """Empty reference (Eq. 3): only tuples holding both occupied and virtual
    MOs give non-zero increments, so the expansion starts at order 2."""
    p, r = hub8
    occ = set(p.occ)
    for t, d in zip(r["tuples"], r["inc"]):
        if set(t) <= occ or not (set(t) & occ):
            assert abs(d) < 1e-12, t
    assert abs(r["e_order"][0]) < 1e-12
    # E_ref of the vacuum reference is the reference-determinant energy
    h, g = p.h1, p.eri
    o = p.occ
    e_det = 2 * sum(h[i, i] for i in o) + sum(2 * g[i, i, j, j] - g[i, j, j, i] for i in o for j in o)
    assert abs(r["e_ref"] - e_det) < 1e-12


def test_recursion_matches_moebius(hub8):
    p, r = hub8
    f = dict(zip(r["tuples"], r["f"]))
    e_m = mbe.moebius_order_sums(r["e_ref"], f, len(p.exp), p.max_order)
    assert np.max(np.abs(np.array(e_m) - np.array(r["e_order"]))) < 1e-10
    # per tuple: Delta eps_T = sum_{U subset T} (-1)^{|T|-|U|} f(U)
    fall = dict(f)
    fall[()] = r["e_ref"]
    for t, d in list(zip(r["tuples"], r["inc"]))[::17]:
        s = sum((-1) ** (len(t) - m) * fall[u] for m in range(len(t) + 1)
                for u in itertools.combinations(t, m))
        assert abs(s - d) < 1e-11


def test_zero_interaction_gives_zero_increments():
    """U = 0: every CASCI equals the reference-determinant energy shifted by
    nothing, so all increments vanish."""
    h, g = W.hubbard_mo(6, 1.0, 0.0)
    p = W.Problem("u0", h, g, 0.0, [0, 1, 2], [], list(range(6)), 6)
    r = mbe.mbe(p, workers=1)
    assert max(abs(d) for d in r["inc"]) < 1e-12


def test_reference_space_expansion_full_order():
    """General reference space (Eq. 1): the full expansion over the rest equals
    the whole-space FCI."""
    h, g = W.hubbard_mo(8, 1.0, 2.0)
    p = W.Problem("h8ref", h, g, 0.0, [0, 1, 2, 3], [3, 4], [0, 1, 2, 5, 6, 7], 6)
    r = mbe.mbe(p, workers=1)
    assert abs(r["e_total"] - fci.casci(h, g, 0.0, p.occ, range(8))) < 1e-10


def test_adjoint_weights_match_moebius():
    tups = mbe.tuples(range(6), 4)
    rng = np.random.default_rng(0)
    g_ref, g_ord = rng.standard_normal(), rng.standard_normal(4)
    w_ref, w = mbe.increment_adjoint(g_ref, g_ord, tups)
    nexp = 6
    exp_ref = g_ref + sum(g_ord[n - 1] * (-1) ** n * math.comb(nexp, n) for n in range(1, 5))
    assert abs(w_ref - exp_ref) < 1e-12
    for t in tups:
        u = len(t)
        exp = sum(g_ord[n - 1] * (-1) ** (n - u) * math.comb(nexp - u, n - u) for n in range(u, 5))
        assert abs(w[t] - exp) < 1e-12


# ------------------------------------------------------------------- RDMs
def test_two_site_rdm_closed_forms():
    gold = _golden("two_site_hubbard.txt")
    h, g = W.hubbard_site(2, 1.0, 2.0)
    e, gamma, Gamma = rdm.casci_rdms(h, g, 0.0, [0], [0, 1])
    assert abs(np.sum(h * gamma) - gold["E_1e"]) < 1e-13
    assert abs(0.5 * np.sum(g * Gamma) - gold["E_2e"]) < 1e-13


@pytest.mark.parametrize("active", [[0, 1, 2, 3, 4, 5], [1, 2, 4], [0, 3, 5]])
def test_rdm_traces_and_energy_reconstruction(active):
    h, g = W.synthetic(6, 5)
    occ = [0, 1, 2]
    e, gamma, Gamma = rdm.casci_rdms(h, g, 0.3, occ, active)
    ne = 2 * len(occ)
    assert abs(np.trace(gamma) - ne) < 1e-12
    assert abs(np.einsum("pprr->", Gamma) - ne * (ne - 1)) < 1e-11
    assert abs(rdm.energy_from_rdms(h, g, 0.3, gamma, Gamma) - e) < 1e-11


def _sym_direction(M, rng):
    vh = rng.standard_normal((M, M))
    vh = vh + vh.T
    vg = rdm.sym8(rng.standard_normal((M,) * 4))
    return vh, vg


def test_mbe_gradient_matches_finite_differences():
    h, g = W.hubbard_mo(6, 1.0, 3.0)
    p = W.Problem("h6", h, g, 0.0, [0, 1, 2], [], list(range(6)), 3)
    rng = np.random.default_rng(1)
    g_ord = rng.standard_normal(3)
    g_ref = 0.7
    dh, dg, _, _ = rdm.mbe_gradient(p, g_ref, g_ord)

    def loss(hh, gg):
        q = W.Problem("h6", hh, gg, 0.0, p.occ, p.ref, p.exp, p.max_order)
        r = mbe.mbe(q, workers=1)
        return g_ref * r["e_ref"] + float(np.dot(g_ord, r["e_order"]))

    step = 1e-5
    for _ in range(3):
        vh, vg = _sym_direction(6, rng)
        fd = (loss(h + step * vh, g + step * vg) - loss(h - step * vh, g - step * vg)) / (2 * step)
        an = np.sum(dh * vh) + np.sum(dg * vg)
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-8


def test_euler_identity():
    """E_MBE is homogeneous of degree one in (h, g):
    <h, dE/dh> + <g, dE/dg> = E_MBE - e_const."""
    h, g = W.hubbard_mo(6, 1.0, 2.5)
    p = W.Problem("h6", h, g, 0.0, [0, 1, 2], [2, 3], [0, 1, 4, 5], 2)
    dh, dg, _, _ = rdm.mbe_gradient(p, 1.0, [1.0, 1.0])
    r = mbe.mbe(p, workers=1)
    assert abs(np.sum(h * dh) + np.sum(g * dg) - r["e_total"]) < 1e-10
