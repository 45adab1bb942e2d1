"""Every CASCI of the two headline expansions against the oracle (needs an
MI355X), in the batched launch configuration that bench.py times.

* Hubbard-16 (6-MO reference, order 4: 385 tuples plus the reference CASCI)
  and synthetic M = 40 ((6e,6o) reference, order 3: 6,579 tuples plus the
  reference CASCI).  The oracle's f(T) of every tuple is stored in
  ``tests/golden/mbe_<name>.txt`` (written by ``make_mbe_goldens.py`` from
  ``oracle/`` only).  Each GPU CASCI energy (the constituent CASCI
  calculations of Eq. 1), each increment (Eq. 2: recomputed from the stored
  energies by the oracle's recursion), each order sum E^(n) and E_total
  (Eq. 1) must agree to 1e-9 E_h.
* The inputs are regenerated from the seeded generators; their sums and norms
  must match the ones stored with the goldens (to rounding: BLAS builds may
  differ in the last bit).
* Davidson residual tolerance: the one bench.py runs each expansion at.  The
  order sums add each CASCI energy with binomial weights (up to C(33,2) = 528
  for an order-1 energy in E^(3) of the 34-orbital expansion), so the
  synthetic M = 40 expansion runs at 3e-7 (E^(3) within 2e-10 of the
  oracle; at 1e-6 it is 2.7e-9 off although every CASCI agrees to 1.3e-12),
  Hubbard-16 at the library default 1e-6 (E^(n) within 1e-10).
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from golden_io import read_mbe_golden as read_golden
from oracle import mbe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _fingerprint(p):
    return [float(np.sum(p.h1)), float(np.sum(p.eri)), float(np.linalg.norm(p.h1)),
            float(np.linalg.norm(p.eri))]


CONV_TOL = {"hubbard16": 1e-6, "synthetic40": 3e-7}


@pytest.mark.parametrize("name", ["hubbard16", "synthetic40"])
def test_every_casci_matches_oracle(name):
    from paper_1910_03527_amd import Context
    p = W.problem(name)
    fp, f_ref, f = read_golden(name)
    for a, b in zip(_fingerprint(p), fp):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), "inputs differ from the goldens' inputs"
    tups = mbe.tuples(p.exp, p.max_order)
    assert sorted(f) == sorted(tups)
    _log("gpu full expansion", name, len(tups) + 1, "CASCIs")
    ctx = Context(0, conv_tol=CONV_TOL[name])
    try:
        r = ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order,
                            want_increments=True)
    finally:
        ctx.close()
    assert abs(r["e_ref"] - f_ref) < 1e-9
    got_f = np.array(r["energies"])
    exp_f = np.array([f[t] for t in tups])
    err_f = np.abs(got_f - exp_f)
    _log("  max |f_GPU - f_oracle|", float(err_f.max()), "at", tups[int(err_f.argmax())])
    assert err_f.max() < 1e-9
    _, dinc = mbe.increments(f_ref, f)
    exp_inc = np.array([dinc[t] for t in tups])
    err_inc = np.abs(np.array(r["increments"]) - exp_inc)
    _log("  max |increment difference|", float(err_inc.max()))
    assert err_inc.max() < 1e-9
    e_order = mbe.order_sums(dinc, p.max_order)
    _log("  E^(n) differences", [r["e_order"][n] - e_order[n] for n in range(p.max_order)])
    for n in range(p.max_order):
        assert abs(r["e_order"][n] - e_order[n]) < 1e-9, n + 1
    assert abs(r["e_total"] - (f_ref + sum(e_order))) < 1e-9


def test_tight_tolerance_synthetic40():
    """The synthetic M = 40 expansion at residual 1e-9: every CASCI converges
    (CASCIs switch to the Olsen correction below residual 1e-7; with the
    P-space correction alone some stagnated below 3e-8), every CASCI energy
    agrees with the oracle's to 1e-11 and the order sums to 1e-9 (at 3e-7 and
    at 1e-9 E^(3) is 1.6e-10 off: the binomially weighted sum of per-CASCI
    differences near the oracle's own Lanczos accuracy, not the residual)."""
    from paper_1910_03527_amd import Context
    name = "synthetic40"
    p = W.problem(name)
    _, f_ref, f = read_golden(name)
    _log("gpu full expansion", name, "at residual 1e-9")
    ctx = Context(0, conv_tol=1e-9)
    try:
        r = ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order,
                            want_increments=True)
        st = dict(ctx.last_stats)
    finally:
        ctx.close()
    _log("  max_iters", st["max_iters"], "first_failed", st["first_failed"])
    assert st["first_failed"] == -1
    assert st["max_iters"] <= 80, st["max_iters"]
    tups = mbe.tuples(p.exp, p.max_order)
    err_f = np.abs(np.array(r["energies"]) - np.array([f[t] for t in tups]))
    _log("  max |f_GPU - f_oracle|", float(err_f.max()))
    assert err_f.max() < 1e-11 and abs(r["e_ref"] - f_ref) < 1e-11
    _, dinc = mbe.increments(f_ref, f)
    e_order = mbe.order_sums(dinc, p.max_order)
    diff = [r["e_order"][n] - e_order[n] for n in range(p.max_order)]
    _log("  E^(n) differences", diff)
    assert max(abs(d) for d in diff) < 1e-9
