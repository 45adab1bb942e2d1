"""RDM backward of the HIP path vs the CPU oracle and finite differences
(needs an MI355X).

Gradients are 8-fold symmetrised for the two-electron integrals (dE/d(pq|rs) =
Gamma/2 averaged over the permutations of (pq|rs)) and symmetric for h, the
convention both sides use.  Tolerances: RDMs 1e-9 absolute; MBE gradients
against the oracle 1e-8 absolute (sums of up to thousands of weighted RDMs,
each converged to a 1e-9 residual); finite differences 1e-6 relative + 1e-8.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fci, rdm as ordm

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
    c = Context(0, conv_tol=1e-9, max_iter=400)
    yield c
    c.close()


@pytest.mark.parametrize("n,na,nb", [(4, 2, 2), (5, 2, 3), (6, 3, 3), (7, 3, 3), (8, 4, 4)])
def test_casci_rdms_match_oracle(ctx, n, na, nb):
    _log("casci rdm", n, na, nb)
    h, g = W.synthetic(n, 500 + n)
    a = fci.string_masks(range(n), na)
    b = fci.string_masks(range(n), nb)
    H = fci.hamiltonian(h, g, 0.0, a, b)
    e, v = fci.lowest(H, want_vec=True)
    gam, Gam = ordm.rdm12(a, b, v / np.linalg.norm(v), n)
    got_e = ctx.casci([_dev(h)], [_dev(g)], na, nb)[0]
    g1, g2 = ctx.casci_rdm()
    g1 = g1[0].cpu().numpy()
    g2 = g2[0].cpu().numpy()
    assert abs(got_e - e) < 1e-9
    assert np.max(np.abs(g1 - 0.5 * (gam + gam.T))) < 1e-9
    assert np.max(np.abs(g2 - ordm.sym8(Gam))) < 1e-9
    # energy reconstruction from the GPU RDMs
    assert abs(np.sum(h * g1) + 0.5 * np.sum(g * g2) - got_e) < 1e-9


def _gpu_grad(ctx, p, gvec):
    ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order, p.e_const)
    dh, dg = ctx.mbe_backward(gvec)
    return dh.cpu().numpy(), dg.cpu().numpy()


SMALL = [
    ("hub6_vacuum", lambda: W.Problem("h6", *W.hubbard_mo(6, 1.0, 3.0), 0.0, [0, 1, 2], [],
                                      list(range(6)), 3)),
    ("hub8_ref2", lambda: W.Problem("h8r", *W.hubbard_mo(8, 1.0, 2.0), 0.0, [0, 1, 2, 3], [3, 4],
                                    [0, 1, 2, 5, 6, 7], 3)),
    ("syn7_ref3", lambda: W.Problem("s7", *W.synthetic(7, 9), 0.0, [0, 1, 2], [1, 2, 3],
                                    [0, 4, 5, 6], 3)),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_mbe_gradient_matches_oracle(ctx, name, make):
    _log("mbe grad", name)
    p = make()
    rng = np.random.default_rng(3)
    gvec = rng.standard_normal(1 + p.max_order)
    dh_o, dg_o, _, _ = ordm.mbe_gradient(p, gvec[0], gvec[1:], workers=min(16, os.cpu_count() or 1))
    dh, dg = _gpu_grad(ctx, p, gvec)
    assert np.max(np.abs(dh - dh_o)) < 1e-8
    assert np.max(np.abs(dg - dg_o)) < 1e-8


def test_reference_rdm_embedding(ctx):
    """Upstream gradient (1, 0, ...): the gradient of E_ref alone, i.e. the
    full-space RDMs of the reference CASCI with its frozen core."""
    _log("ref embedding")
    p = SMALL[1][1]()
    e, gam, Gam = ordm.casci_rdms(p.h1, p.eri, 0.0, p.occ, p.ref)
    dh, dg = _gpu_grad(ctx, p, [1.0] + [0.0] * p.max_order)
    assert np.max(np.abs(dh - 0.5 * (gam + gam.T))) < 1e-9
    assert np.max(np.abs(dg - 0.5 * ordm.sym8(Gam))) < 1e-9


@pytest.fixture(scope="module")
def hub12_grad(ctx):
    p = W.problem("hubbard12")
    gvec = np.array([0.3, 1.0, -0.7, 1.3, 0.5, -1.1, 0.9])
    dh, dg = _gpu_grad(ctx, p, gvec)
    return p, gvec, dh, dg


def test_hubbard12_gradient_matches_oracle(ctx, hub12_grad):
    _log("hubbard12 grad vs oracle")
    p, gvec, dh, dg = hub12_grad
    dh_o, dg_o, _, _ = ordm.mbe_gradient(p, gvec[0], gvec[1:], workers=min(16, os.cpu_count() or 1))
    assert np.max(np.abs(dh - dh_o)) < 1e-8
    assert np.max(np.abs(dg - dg_o)) < 1e-8
    # each orbit of the integrals' 8-fold symmetry gets one value (and dh one
    # per p >= q), so the gradients are exactly symmetric
    assert np.array_equal(dh, dh.T)
    for perm in ((1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)):
        assert np.array_equal(dg, dg.transpose(perm)), perm


def test_hubbard12_gradient_finite_differences(ctx, hub12_grad):
    """Central differences (step 1e-5) along random symmetric directions."""
    _log("hubbard12 FD")
    p, gvec, dh, dg = hub12_grad
    rng = np.random.default_rng(11)

    def loss(h, g):
        r = ctx.mbe_forward(_dev(h), _dev(g), p.occ, p.ref, p.exp, p.max_order, p.e_const)
        return gvec[0] * r["e_ref"] + float(np.dot(gvec[1:], r["e_order"]))

    step = 1e-5
    for _ in range(4):
        vh = rng.standard_normal((12, 12))
        vh = vh + vh.T
        vg = ordm.sym8(rng.standard_normal((12,) * 4))
        fd = (loss(p.h1 + step * vh, p.eri + step * vg)
              - loss(p.h1 - step * vh, p.eri - step * vg)) / (2 * step)
        an = float(np.sum(dh * vh) + np.sum(dg * vg))
        assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-8, (an, fd)


def _orbits(M):
    """Unique elements of a symmetric M x M matrix and of an 8-fold symmetric
    M^4 tensor, each with the index arrays of all its symmetric copies."""
    hs = []
    for p in range(M):
        for q in range(p, M):
            hs.append(sorted({(p, q), (q, p)}))
    pairs = [(p, q) for p in range(M) for q in range(p, M)]
    gs = []
    for i, (p, q) in enumerate(pairs):
        for (r, s) in pairs[i:]:
            gs.append(sorted({(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                              (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}))
    return hs, gs


def test_hubbard12_gradient_fd_every_element(ctx, hub12_grad):
    """Central differences (step 1e-5) along every unique element of h (78)
    and of (pq|rs) (3,081 orbits of the 8-fold symmetry), each perturbed in all
    its symmetric copies, against the analytic dL/d(element) summed over the
    copies.  Per element: |an - fd| <= 1e-6 |fd| + 2e-7.  The floor is the FD
    noise: L adds the energies of 2,510 CASCIs with alternating binomial
    weights (Eq. 2), so its rounding is 1e-12 to 2e-12 E_h (it depends on
    how often the Davidson subspace restarts), and divided by the step that
    is 1e-7 to 2e-7; elements that vanish by the chain's reflection
    symmetry show only that noise.  Over all elements the normwise relative
    error must stay below 1e-6."""
    _log("hubbard12 FD over every unique element")
    p, gvec, dh, dg = hub12_grad
    M = p.norb
    step = 1e-5
    h0 = _dev(p.h1)
    g0 = _dev(p.eri)

    def loss(h, g):
        r = ctx.mbe_forward(h, g, p.occ, p.ref, p.exp, p.max_order, p.e_const)
        return gvec[0] * r["e_ref"] + float(np.dot(gvec[1:], r["e_order"]))

    hs, gs = _orbits(M)
    assert len(hs) == 78 and len(gs) == 3081
    an_all, fd_all = [], []
    for kind, orbits, base, grad in (("h", hs, h0, dh), ("g", gs, g0, dg)):
        for k, orbit in enumerate(orbits):
            idx = tuple(torch.tensor(x, device="cuda") for x in zip(*orbit))
            xp, xm = base.clone(), base.clone()
            xp[idx] += step
            xm[idx] -= step
            if kind == "h":
                fd = (loss(xp, g0) - loss(xm, g0)) / (2 * step)
            else:
                fd = (loss(h0, xp) - loss(h0, xm)) / (2 * step)
            an = float(sum(grad[e] for e in orbit))
            an_all.append(an)
            fd_all.append(fd)
            assert abs(an - fd) <= 1e-6 * abs(fd) + 2e-7, (kind, orbit[0], an, fd)
            if kind == "g" and k % 1000 == 0:
                _log("  orbit", k, "of", len(orbits))
    an_all, fd_all = np.array(an_all), np.array(fd_all)
    rel = np.linalg.norm(an_all - fd_all) / np.linalg.norm(fd_all)
    big = np.abs(fd_all) > 1e-2
    _log("  normwise relative error", rel, "; largest relative error of the",
         int(big.sum()), "elements above 1e-2:",
         float(np.max(np.abs(an_all - fd_all)[big] / np.abs(fd_all[big]))),
         "; largest |an - fd| of the others:", float(np.max(np.abs(an_all - fd_all)[~big])))
    assert rel < 1e-6


def test_euler_identity(ctx, hub12_grad):
    """L is homogeneous of degree one in (h, g): <h, dL/dh> + <g, dL/dg> = L."""
    p, gvec, dh, dg = hub12_grad
    r = ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order)
    L = gvec[0] * r["e_ref"] + float(np.dot(gvec[1:], r["e_order"]))
    assert abs(np.sum(p.h1 * dh) + np.sum(p.eri * dg) - L) < 1e-9


def test_autograd_function(ctx):
    _log("autograd")
    from paper_1910_03527_amd import MBEEnergy
    p = SMALL[0][1]()
    h = _dev(p.h1).requires_grad_(True)
    g = _dev(p.eri).requires_grad_(True)
    out = MBEEnergy.apply(h, g, ctx, p.occ, p.ref, p.exp, p.max_order)
    out.sum().backward()
    dh_o, dg_o, _, _ = ordm.mbe_gradient(p, 1.0, [1.0] * p.max_order)
    assert np.max(np.abs(h.grad.cpu().numpy() - dh_o)) < 1e-8
    assert np.max(np.abs(g.grad.cpu().numpy() - dg_o)) < 1e-8
