"""Pins of the screened-expansion oracle (``oracle/screen.py``).

* Eq. 4 with the paper's parameters (T_init = 1e-10 E_h, M_init = 3,
  a = 5.0): zero below M_init, T_init at M_init, times a per extra MO.
* The order-by-order spawning, which the oracle runs per parent as the
  paper words it, against the same rule restated child by child by brute
  force over all subsets (a child C is spawned iff C has two different
  order-k sub-tuples P and Q, P computed and Q computed with |Delta eps_Q|
  above T_tup(Q): P is the parent, Q = S + c), on random increment tables.
* A hand-built increment table on which this rule and the looser "any
  computed order-k sub-tuple above its threshold" rule spawn different
  children (a child whose only computed sub-tuple is significant is not
  spawned: that sub-tuple would be its own parent).
* T_init = 0: every tuple with a non-vanishing increment survives, so the
  screened expansion equals the full one (the oracle's Eq. 2 recursion).
* Telescoping: when the whole expansion space X is computed, E_total = f(X)
  whatever subset of sub-tuples was kept (the increments over the computed
  set sum to eps_X).
* Monotonicity in the threshold, and the large-threshold limit, where only
  sub-tuples below M_init (threshold 0) spawn.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import fci, mbe, screen


def test_threshold_eq4_paper_parameters():
    occ = {0, 1, 2, 3, 4}
    t = lambda tup: screen.threshold(tup, occ, 1e-10, 3, 5.0)
    assert t((0,)) == 0.0 and t((0, 5)) == 0.0 and t((0, 1, 5, 6)) == 0.0
    assert t((0, 1, 2)) == 1e-10            # M_tup = 3 occupied
    assert t((5, 6, 7, 0)) == 1e-10          # M_tup = 3 virtual
    assert t((0, 1, 2, 3, 5)) == pytest.approx(5e-10, rel=1e-15)
    assert t((0, 1, 2, 3, 4, 5)) == pytest.approx(2.5e-9, rel=1e-15)
    assert screen.threshold((0, 1, 2, 3), occ, 1e-10, 3, 2.5) == pytest.approx(2.5e-10, rel=1e-15)
    assert screen.m_tup((0, 1, 5), occ) == 2 and screen.m_tup((5, 6, 7, 8), occ) == 4


def _brute_children(prev, exp, occ, ref, t_init, m_init, a):
    """The per-parent rule, child by child: C (not a structural zero) is
    spawned iff two different order-k sub-tuples P, Q of C exist with P
    computed (the parent) and Q computed above its own threshold."""
    k = len(next(iter(prev)))
    out = []
    for c in itertools.combinations(sorted(exp), k + 1):
        if screen.structural_zero(c, occ, ref):
            continue
        subs = list(itertools.combinations(c, k))
        sig = [q for q in subs
               if q in prev and abs(prev[q]) > screen.threshold(q, occ, t_init, m_init, a)]
        if any(p in prev and p != q for p in subs for q in sig):
            out.append(c)
    return out


def test_spawn_per_parent_differs_from_any_subtuple_rule():
    """Hand-built order-2 table (reference space non-empty, so no structural
    zeros; M_init = 3 puts every pair's threshold at 0): (0,1) and (2,3)
    significant, (2,4) computed with a zero increment.  Any-sub-tuple rule:
    the six supersets of (0,1) and (2,3).  Per parent: only (2,3,4), whose
    parent (2,4) forms (2,3) = {2} + 3; the supersets of (0,1) and (2,3)
    have no other computed pair, so no parent forms the significant pair."""
    exp = [0, 1, 2, 3, 4]
    occ = {0, 1}
    ref = [5]
    prev = {(0, 1): 1e-3, (2, 3): -2e-3, (2, 4): 0.0}
    got = screen.spawn(prev, exp, occ, ref, 1e-10, 3, 5.0)
    assert got == [(2, 3, 4)]
    loose = sorted({tuple(sorted(s + (c,))) for s, d in prev.items() if d != 0.0
                    for c in exp if c not in s})
    assert loose == [(0, 1, 2), (0, 1, 3), (0, 1, 4), (0, 2, 3), (1, 2, 3), (2, 3, 4)]
    assert got != loose
    # the parent's own increment plays no part: make (2,4) huge and (2,3) zero
    prev2 = {(0, 1): 1e-3, (2, 3): 0.0, (2, 4): 5.0}
    assert screen.spawn(prev2, exp, occ, ref, 1e-10, 3, 5.0) == [(2, 3, 4)]
    # thresholds are those of the tested tuple S + c: at order 3 with
    # M_init = 2, T_tup = t_init * a^(M_tup - 2)
    prev3 = {(0, 2, 3): 3e-6, (0, 2, 4): 1e-9}
    occ3 = {0, 1, 2}
    # (0,2,3): M_tup 2 -> T = 1e-6 -> significant; (0,2,4): T = 1e-6 -> not
    assert screen.spawn(prev3, exp, occ3, ref, 1e-6, 2, 10.0) == [(0, 2, 3, 4)]
    # (0,2,3) below its threshold now: nothing
    assert screen.spawn(prev3, exp, occ3, ref, 1e-5, 2, 10.0) == []


@pytest.mark.parametrize("seed", range(6))
def test_spawn_matches_child_by_child_definition(seed):
    rng = np.random.default_rng(seed)
    exp = list(range(9))
    occ = {0, 1, 2, 3}
    ref = [] if seed % 2 == 0 else [9]
    k = 2 + seed % 3
    prev = {}
    for s in itertools.combinations(exp, k):
        if screen.structural_zero(s, occ, ref) or rng.random() < 0.3:
            continue
        prev[s] = float(rng.choice([0.0, 1e-12, 1e-9, 1e-6, -3e-8, 2e-3]))
    for t_init, a in [(0.0, 5.0), (1e-9, 5.0), (1e-7, 2.5)]:
        got = screen.spawn(prev, exp, occ, ref, t_init, 3, a)
        assert got == _brute_children(prev, exp, occ, ref, t_init, 3, a)


def _small_ref_problem():
    h1, g = W.synthetic(9, 41)
    return W.Problem("s9", h1, g, 0.0, [0, 1, 2, 3], [3, 4], [0, 1, 2, 5, 6, 7, 8], 3)


@pytest.mark.parametrize("name", ["hubbard8", "ref"])
def test_zero_threshold_equals_full_expansion(name):
    if name == "hubbard8":
        p = W.problem("hubbard8")
        k = 5
    else:
        p = _small_ref_problem()
        k = 3
    full = mbe.mbe(p, max_order=k, workers=4)
    scr = screen.screened_mbe(p, 0.0, 3, 5.0, max_order=k, workers=4)
    assert abs(scr["e_ref"] - full["e_ref"]) < 1e-12
    assert np.max(np.abs(np.array(scr["e_order"]) - np.array(full["e_order"]))) < 1e-10
    # every non-structural tuple was computed, with the full expansion's increment
    finc = dict(zip(full["tuples"], full["inc"]))
    for lvl in scr["per_order"]:
        for t, d in lvl:
            assert abs(d - finc[t]) < 1e-10
    ncomp = sum(len(l) for l in scr["per_order"])
    nfull = sum(1 for t in full["tuples"]
                if not screen.structural_zero(t, set(p.occ), p.ref))
    assert ncomp == nfull


def test_telescoping_to_whole_space():
    p = W.problem("hubbard8")
    exact = fci.casci(p.h1, p.eri, 0.0, p.occ, range(8))
    r = screen.screened_mbe(p, 1e-3, 3, 5.0, workers=4)
    # some tuples were screened away, yet the whole space was computed
    assert sum(len(l) for l in r["per_order"]) < 254 - 30
    assert r["per_order"][7] and r["per_order"][7][0][0] == tuple(range(8))
    assert abs(r["e_total"] - exact) < 1e-10


def test_threshold_monotonicity_and_large_limit():
    p = W.problem("hubbard8")
    occ = set(p.occ)
    sets = []
    for t_init in [0.0, 1e-4, 1e-3, 1e3]:
        r = screen.screened_mbe(p, t_init, 3, 5.0, max_order=6, workers=4)
        sets.append([set(t for t, _ in l) for l in r["per_order"]])
    for a, b in zip(sets, sets[1:]):
        for x, y in zip(a, b):
            assert y <= x
    # T_init = 1e3: only tuples with M_tup < 3 (threshold 0) are significant,
    # so from order 2 on the computed tuples are exactly the children C with
    # a computed order-k sub-tuple P and another one, Q != P, with M_tup < 3
    # and a non-zero increment
    big = screen.screened_mbe(p, 1e3, 3, 5.0, max_order=6, workers=4)
    for k in range(2, 6):
        prev = dict(big["per_order"][k - 1])
        cur = set(t for t, _ in big["per_order"][k])
        exp_children = set()
        for c in itertools.combinations(sorted(p.exp), k + 1):
            if screen.structural_zero(c, occ, p.ref):
                continue
            subs = [s for s in itertools.combinations(c, k) if s in prev]
            if any(q != s and screen.m_tup(q, occ) < 3 and prev[q] != 0.0
                   for s in subs for q in subs):
                exp_children.add(c)
        assert cur == exp_children
