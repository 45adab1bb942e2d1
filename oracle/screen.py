"""Oracle of the screened, order-by-order expansion (the tuple-screening rule
and the threshold of Eq. 4).  Test infrastructure only.

The paper states the rule in words; this module takes these readings:

* A tuple T is a set of expansion orbitals.  M_tup(T) = max(M_occ, M_virt),
  the larger of its numbers of occupied MOs (doubly occupied in the reference
  determinant) and of virtual MOs.
* Eq. 4: T_tup = 0 when M_tup < M_init, else T_init * a^(M_tup - M_init).
* Order 1 holds every expansion orbital.  Spawning follows the per-parent
  rule stated with Eq. 4: for a computed parent P of order k and a candidate
  orbital c of X not in P, the order-k tuples S + c are formed for every
  (k-1)-subtuple S of P (the parent itself is not among them); the child
  P + c is spawned when |Delta eps| of any of them exceeds that tuple's own
  threshold T_tup.  A tuple S + c that was never computed has no increment
  and cannot trigger a spawn.  Every computed tuple of order k acts as a
  parent and every orbital of X outside it as a candidate; the children of
  order k+1 are the union over parents.  (Restricting candidates to orbitals
  above the parent's last one would make the result depend on the orbital
  numbering, which the paper does not make part of the rule.)
* With an empty reference space (Eq. 3) a tuple made only of occupied or
  only of virtual MOs has a vanishing increment for a structural reason (its
  CASCI is the reference determinant itself).  Such tuples are never
  computed and count as Delta eps = 0 (they are no parents and trigger no
  spawn).  The mixed pairs, whose order-1 sub-tuples are all of that kind,
  have no computed parent; they form the first order computed, all of them.
* Increments follow Eq. 2 over the computed sub-tuples: Delta eps_T = eps_T
  minus the increments of its computed proper non-empty sub-tuples (a
  sub-tuple never computed contributes 0).  E^(k) is the sum of the order-k
  increments and E_total = E_ref + sum_k E^(k) (Eq. 1).
"""
from __future__ import annotations

import itertools
import os

from . import mbe as _mbe


def m_tup(t, occ):
    """max(number of occupied, number of virtual) MOs of tuple ``t``."""
    o = sum(1 for p in t if p in occ)
    return max(o, len(t) - o)


def threshold(t, occ, t_init, m_init, a):
    """T_tup of Eq. 4 for tuple ``t``."""
    m = m_tup(t, occ)
    return 0.0 if m < m_init else t_init * a ** (m - m_init)


def structural_zero(t, occ, ref):
    """True when the increment of ``t`` vanishes by construction: empty
    reference space and a tuple of only occupied or only virtual MOs."""
    if len(ref) != 0:
        return False
    o = sum(1 for p in t if p in occ)
    return o == 0 or o == len(t)


def spawn(prev, exp, occ, ref, t_init, m_init, a):
    """Children of order k+1 from the computed order-k parent tuples ``prev``
    (dict tuple -> increment), lexicographically sorted.  Per parent P and
    candidate orbital c: the tuples S + c, S every (k-1)-subtuple of P, are
    tested against their own thresholds; one above spawns P + c."""
    occ = set(occ)
    x = sorted(exp)
    out = set()
    for par in prev:
        k = len(par)
        for c in x:
            if c in par:
                continue
            child = tuple(sorted(par + (c,)))
            if child in out or structural_zero(child, occ, ref):
                continue
            for s in itertools.combinations(par, k - 1):
                q = tuple(sorted(s + (c,)))
                if q in prev and abs(prev[q]) > threshold(q, occ, t_init, m_init, a):
                    out.add(child)
                    break
    return sorted(out)


def first_level(exp, occ, ref):
    """The first tuples to compute: order 1, or with an empty reference space
    (where every order-1 tuple is a structural zero) the mixed pairs."""
    occ = set(occ)
    x = sorted(exp)
    one = [(p,) for p in x if not structural_zero((p,), occ, ref)]
    if one:
        return 1, one
    return 2, [t for t in itertools.combinations(x, 2) if not structural_zero(t, occ, ref)]


def screened_mbe(prob, t_init, m_init, a, max_order=None, workers=None):
    """Screened expansion of a ``workloads.Problem``.  Returns E_ref, E^(k),
    E_total and, per order, the computed tuples and their increments."""
    kmax = prob.max_order if max_order is None else max_order
    if workers is None:
        workers = os.cpu_count() or 1
    occ = set(prob.occ)
    osym = getattr(prob, "orbsym", None)
    f_ref = _mbe.tuple_energies(prob.h1, prob.eri, prob.e_const, prob.occ, prob.ref, [()], 1,
                                osym)[0]
    inc = {}
    e_order = [0.0] * kmax
    per_order = [[] for _ in range(kmax)]
    k, level = first_level(prob.exp, occ, prob.ref)
    while k <= kmax and level:
        f = _mbe.tuple_energies(prob.h1, prob.eri, prob.e_const, prob.occ, prob.ref, level, workers,
                                osym)
        cur = {}
        for t, ft in zip(level, f):
            d = ft - f_ref
            for m in range(1, len(t)):
                for u in itertools.combinations(t, m):
                    d -= inc.get(u, 0.0)
            cur[t] = d
        inc.update(cur)
        e_order[k - 1] = sum(cur[t] for t in level)
        per_order[k - 1] = [(t, cur[t]) for t in level]
        if k == kmax:
            break
        level = spawn(cur, prob.exp, occ, prob.ref, t_init, m_init, a)
        k += 1
    return {
        "e_ref": f_ref,
        "e_order": e_order,
        "e_total": f_ref + sum(e_order),
        "per_order": per_order,
    }
