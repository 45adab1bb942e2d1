"""The HIP path at the benchmark workloads' full sizes, in the batched launch
configuration bench.py times (needs an MI355X).

* Hubbard-16 (6-MO reference, order 4, 386 CASCIs) and synthetic M=40
  ((6e,6o) reference, order 3, 6,580 CASCIs): the reference CASCI and the first
  tuple of every (order, occupied-count) bucket are solved by the oracle one
  by one; energies must agree to 1e-9 Eh.  The whole expansion must satisfy
  the order-sum identity against the reported increments.
* 8 x CAS(14e,14o) (11,778,624 determinants each): the energies of the
  instances in ``tests/golden/casci_large.txt`` (the oracle's matrix-free
  Slater-Condon Lanczos, ``make_casci_goldens.py``) to 1e-9 E_h; every GPU
  eigenpair row by row against the oracle's Slater-Condon rows (sigma_I =
  E c_I on sampled determinants), and the RDMs against the invariants
  tr gamma = N, sum_pr Gamma_pprr = N(N-1) and E = sum h gamma + 1/2 sum g
  Gamma.
"""
import itertools
import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads as W
from golden_io import read_large_goldens
from oracle import fci

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _sample(prob):
    occ = set(prob.occ)
    xo = sorted(p for p in prob.exp if p in occ)
    xv = sorted(p for p in prob.exp if p not in occ)
    out = [()]
    for n in range(1, prob.max_order + 1):
        for a in range(0, n + 1):
            if math.comb(len(xo), a) * math.comb(len(xv), n - a):
                out.append(tuple(sorted(xo[:a] + xv[:n - a])))
                # and the last tuple of the bucket (ragged ends of the index space)
                out.append(tuple(sorted(xo[len(xo) - a:] + xv[len(xv) - (n - a):])))
    return sorted(set(out), key=lambda t: (len(t), t))


def _oracle_job(args):
    h, g, occ, active = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return fci.casci(h, g, 0.0, occ, active)


@pytest.mark.parametrize("name", ["hubbard16", "synthetic40"])
def test_expansion_sampled_against_oracle(name):
    from paper_1910_03527_amd import Context
    p = W.problem(name)
    tups = _sample(p)
    _log("oracle", name, len(tups), "CASCIs")
    jobs = [(p.h1, p.eri, list(p.occ), sorted(set(p.ref) | set(t))) for t in tups]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        ref = dict(zip(tups, ex.map(_oracle_job, jobs)))
    _log("gpu", name)
    ctx = Context(0)
    try:
        r = ctx.mbe_forward(_dev(p.h1), _dev(p.eri), p.occ, p.ref, p.exp, p.max_order,
                            want_increments=True)
    finally:
        ctx.close()
    allt = list(itertools.chain.from_iterable(
        itertools.combinations(sorted(p.exp), n) for n in range(1, p.max_order + 1)))
    idx = {t: i for i, t in enumerate(allt)}
    assert abs(r["e_ref"] - ref[()]) < 1e-9
    for t in tups[1:]:
        assert abs(r["energies"][idx[t]] - ref[t]) < 1e-9, t
    # E^(n) is the sum of the order-n increments; E_total = E_ref + sum E^(n)
    inc = np.array(r["increments"])
    off = 0
    for n in range(1, p.max_order + 1):
        cnt = math.comb(len(p.exp), n)
        assert abs(np.sum(inc[off:off + cnt]) - r["e_order"][n - 1]) < 1e-10
        off += cnt
    assert abs(r["e_ref"] + sum(r["e_order"]) - r["e_total"]) < 1e-10


def test_cas14_batch_eigenpairs_and_rdms():
    from paper_1910_03527_amd import Context
    probs = [W.problem("cas14", i) for i in range(8)]
    ctx = Context(0)
    try:
        _log("gpu cas14 x8")
        e, cis = ctx.casci([_dev(p.h1) for p in probs], [_dev(p.eri) for p in probs], 7, 7,
                           want_ci=True)
        st = ctx.last_stats
        _log("stats", st)
        g1, g2 = ctx.casci_rdm()
        g1 = g1.cpu().numpy()
        g2 = g2.cpu().numpy()
    finally:
        ctx.close()
    golden = read_large_goldens()
    for i in range(8):
        key = f"cas14_{i}"
        if key in golden:
            _log("  instance", i, "GPU", e[i], "oracle", golden[key])
            assert abs(e[i] - golden[key]) < 1e-9, (i, e[i], golden[key])
    assert "cas14_0" in golden
    a = fci.string_masks(range(14), 7)
    rng = np.random.default_rng(7)
    for i, p in enumerate(probs):
        c = cis[i].cpu().numpy()
        assert abs(np.linalg.norm(c) - 1.0) < 1e-12
        # rows with large and with random weight
        rows = np.unique(np.concatenate([np.argsort(-np.abs(c))[:24],
                                         rng.choice(len(c), 24, replace=False)]))
        sig = fci.sigma_rows(p.h1, p.eri, 0.0, a, a, c, rows)
        assert np.max(np.abs(sig - e[i] * c[rows])) < 2e-6, i
        assert abs(np.trace(g1[i]) - 14.0) < 1e-9
        assert abs(np.einsum("pprr->", g2[i]) - 14.0 * 13.0) < 1e-8
        erec = np.sum(p.h1 * g1[i]) + 0.5 * np.sum(p.eri * g2[i])
        assert abs(erec - e[i]) < 1e-9, (i, erec, e[i])
