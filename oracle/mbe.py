"""Oracle many-body expansion (Eq. 1, Eq. 2, Eq. 3).  Test infrastructure only.

Tuples of expansion orbitals are enumerated order by order in lexicographic
order of the sorted tuple (order n = number of expansion orbitals, so the
first term of Eq. 1 after E_ref is order 1).  For every tuple T the CASCI of
R u T gives f(T); eps_T = f(T) - E_ref with E_ref = f(()) the CASCI of R
alone.  The increments follow Eq. 2 literally: eps_T minus the increments of
every proper non-empty sub-tuple (order-1 increments are the eps_p
themselves).  E^(n) sums the order-n increments and the estimate is
E_ref + sum_n E^(n) (Eq. 1).  With R empty this is Eq. 3: f(()) is the
reference-determinant energy and the expansion starts contributing at
order 2.
"""
from __future__ import annotations

import itertools
import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import fci


def tuples(expansion, max_order):
    """All tuples of 1..max_order expansion orbitals, order by order,
    lexicographic within an order."""
    x = sorted(int(p) for p in expansion)
    out = []
    for n in range(1, max_order + 1):
        out.extend(itertools.combinations(x, n))
    return out


def _casci(h, g, e_const, occ, active, orbsym):
    if orbsym is None:
        return fci.casci(h, g, e_const, occ, active)
    from . import sym
    return sym.casci(h, g, e_const, occ, active, orbsym, 0)


def _solve_one(args):
    h, g, e_const, occ, active, orbsym = args
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return _casci(h, g, e_const, occ, active, orbsym)
    except ImportError:  # pragma: no cover
        return _casci(h, g, e_const, occ, active, orbsym)


def tuple_energies(h, g, e_const, occ, ref, tups, workers=1, orbsym=None):
    """f(T) for T in ``tups`` (the empty tuple gives E_ref).  With ``orbsym``
    (irrep labels of the MOs) each CASCI is solved in the irrep of the
    closed-shell reference determinant, the totally symmetric one."""
    jobs = [(h, g, e_const, list(occ), sorted(set(ref) | set(t)), orbsym) for t in tups]
    if workers <= 1 or len(jobs) < 4:
        return [_solve_one(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_solve_one, jobs, chunksize=max(1, len(jobs) // (8 * workers))))


def increments(f_ref, f):
    """Eq. 2 by recursion.  ``f`` maps tuple -> CASCI energy for every tuple
    up to the maximum order; returns (eps, dinc) dictionaries."""
    eps = {t: f[t] - f_ref for t in f}
    dinc = {}
    for t in sorted(f, key=lambda u: (len(u), u)):
        d = eps[t]
        for m in range(1, len(t)):
            for u in itertools.combinations(t, m):
                d -= dinc[u]
        dinc[t] = d
    return eps, dinc


def order_sums(dinc, max_order):
    """E^(n) = sum of the order-n increments (Eq. 1), summed in tuple order."""
    e = [0.0] * max_order
    for t in sorted(dinc, key=lambda u: (len(u), u)):
        e[len(t) - 1] += dinc[t]
    return e


def mbe(prob, max_order=None, workers=None):
    """Full oracle expansion of a ``workloads.Problem``.

    Returns a dict with E_ref, E_order [k], E_total, and per-tuple f, eps and
    increments (lexicographic tuple order)."""
    k = prob.max_order if max_order is None else max_order
    if workers is None:
        workers = os.cpu_count() or 1
    tups = tuples(prob.exp, k)
    energies = tuple_energies(prob.h1, prob.eri, prob.e_const, prob.occ, prob.ref,
                              [()] + tups, workers, getattr(prob, "orbsym", None))
    f_ref = energies[0]
    f = dict(zip(tups, energies[1:]))
    eps, dinc = increments(f_ref, f)
    e_order = order_sums(dinc, k)
    return {
        "e_ref": f_ref,
        "e_order": e_order,
        "e_total": f_ref + sum(e_order),
        "tuples": tups,
        "f": [f[t] for t in tups],
        "eps": [eps[t] for t in tups],
        "inc": [dinc[t] for t in tups],
    }


def moebius_order_sums(f_ref, f, nexp, max_order):
    """Closed form of the order sums: E^(n) = sum_{|U|<=n} (-1)^(n-|U|)
    C(M_exp-|U|, n-|U|) f(U), with f(()) = E_ref.  Independent of the
    recursion; used to cross-check it."""
    out = []
    for n in range(1, max_order + 1):
        s = (-1) ** n * math.comb(nexp, n) * f_ref
        for t, ft in f.items():
            u = len(t)
            if u <= n:
                s += (-1) ** (n - u) * math.comb(nexp - u, n - u) * ft
        out.append(s)
    return out


def increment_adjoint(g_ref, g_order, tups):
    """Adjoint of the Eq. 2 recursion: d(g_ref E_ref + sum_n g_n E^(n))/d f(U)
    for U = () and every tuple, by reverse-mode through the recursion."""
    bar_inc = {t: float(g_order[len(t) - 1]) for t in tups}
    bar_eps = {}
    for t in sorted(tups, key=lambda u: (len(u), u), reverse=True):
        b = bar_inc[t]
        bar_eps[t] = b
        for m in range(1, len(t)):
            for u in itertools.combinations(t, m):
                bar_inc[u] -= b
    w_ref = float(g_ref) - sum(bar_eps.values())
    return w_ref, bar_eps
