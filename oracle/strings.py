"""Oracle alpha/beta strings and single-excitation link tables (pure Python,
small cases).  Test infrastructure only.

A string of ``nelec`` electrons in ``norb`` active orbitals is a bitmask;
strings are listed in ascending integer order and a string's address is its
position in that list (found here by searching the list, not by formula).

The link table of string I lists, for every one-body operator
E_pq = a+_p a_q (one spin) that does not annihilate I, the entry
(p, q, address of the result, sign), in this canonical order:
  1. the diagonal entries (o, o, I, +1) for o in I ascending;
  2. for q in I ascending, for p not in I ascending: (p, q, J, sign) where
     a+_p a_q |I> = sign |J>.
The sign is obtained by applying a_q then a+_p with the occupation-number
definition ((-1)^(occupied orbitals of lower index) per operator).
"""
from __future__ import annotations

import itertools


def strings(norb, nelec):
    out = []
    for comb in itertools.combinations(range(norb), nelec):
        m = 0
        for o in comb:
            m |= 1 << o
        out.append(m)
    return sorted(out)


def _apply(op, orb, mask):
    """Apply a (op='a') or a+ (op='c') on orbital ``orb``: (sign, mask) or (0, None)."""
    below = bin(mask & ((1 << orb) - 1)).count("1")
    sign = -1 if below % 2 else 1
    occ = (mask >> orb) & 1
    if op == "a":
        if not occ:
            return 0, None
        return sign, mask & ~(1 << orb)
    if occ:
        return 0, None
    return sign, mask | (1 << orb)


def epq(p, q, mask):
    """a+_p a_q |mask> = sign |result>, or (0, None)."""
    s1, m1 = _apply("a", q, mask)
    if not s1:
        return 0, None
    s2, m2 = _apply("c", p, m1)
    if not s2:
        return 0, None
    return s1 * s2, m2


def link_table(norb, nelec):
    """[nstr][nlink] lists of (p, q, J, sign) in the canonical order."""
    strs = strings(norb, nelec)
    addr = {m: i for i, m in enumerate(strs)}
    table = []
    for m in strs:
        occ = [o for o in range(norb) if m >> o & 1]
        vir = [o for o in range(norb) if not m >> o & 1]
        row = [(o, o, addr[m], 1) for o in occ]
        for q in occ:
            for p in vir:
                s, r = epq(p, q, m)
                row.append((p, q, addr[r], s))
        table.append(row)
    return table
