"""Write oracle energies of CASCIs too large for a stored Hamiltonian to
``tests/golden/casci_large.txt``.

Calls only ``oracle/`` and ``workloads/``: the matrix-free Slater-Condon
operator of ``oracle.direct`` with ARPACK Lanczos (tolerance 1e-13 relative
to the eigenvalue).  Cases:

* ``cas14_0``: CAS(14e,14o) of the synthetic generator, M = 14, seed 1 (the
  first of the eight CAS(14,14) instances; 11,778,624 determinants, the size
  of the paper's largest Hubbard CASCI in the Fig. 2 discussion);
* ``cas12_21``, ``cas12_22``: CAS(12e,12o), seeds 21 and 22 (853,776
  determinants, about the size of the benzene final-order CASCI in the Fig. 4
  discussion).

Usage: ``python tests/golden/make_casci_goldens.py [--threads N] [names]``.
CAS(14,14) takes about half an hour on 8 cores.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import direct, fci  # noqa: E402

PATH = os.path.join(HERE, "casci_large.txt")


def case(name):
    """(h1, eri, occupied, active) of a named case."""
    if name.startswith("cas14_"):
        p = W.problem("cas14", int(name[6:]))
        return p.h1, p.eri, p.occ, p.ref
    if name.startswith("cas12_"):
        h, g = W.synthetic(12, int(name[6:]))
        return h, g, list(range(6)), list(range(12))
    raise KeyError(name)


def read():
    """name -> (energy, fingerprint tuple) of the stored cases."""
    out = {}
    if not os.path.exists(PATH):
        return out
    with open(PATH) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = line.split()
            out[w[0]] = (float(w[1]), tuple(float(x) for x in w[2:]))
    return out


def fingerprint(h, g):
    return (float(np.sum(h)), float(np.sum(g)), float(np.linalg.norm(g)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["cas12_21", "cas12_22", "cas14_0"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    rows = read()
    for name in a.names:
        h, g, occ, act = case(name)
        sa, sb = fci.casci_space(occ, act)
        t0 = time.time()
        H = direct.DirectHamiltonian(h, g, 0.0, sa, sb, a.threads)
        e = direct.lowest(H, tol=1e-13)
        wall = time.time() - t0
        print(f"{name}: {H.n} determinants, E = {e:.15f}, {H.nmatvec} sigma, {wall:.0f} s "
              f"on {a.threads} threads", flush=True)
        H.close()
        rows[name] = (e, fingerprint(h, g))
        with open(PATH, "w") as f:
            f.write("# Oracle lowest eigenvalues (E_h) of large CASCIs: matrix-free Slater-Condon\n")
            f.write("# sigma (oracle/direct.py) and ARPACK Lanczos, tolerance 1e-13 relative.\n")
            f.write("# Written by tests/golden/make_casci_goldens.py from oracle/ and workloads/.\n")
            f.write("# name energy sum(h1) sum(eri) |eri|\n")
            for k in sorted(rows):
                en, fp = rows[k]
                f.write(f"{k} {en:.17g} " + " ".join(f"{x:.17g}" for x in fp) + "\n")


if __name__ == "__main__":
    main()
