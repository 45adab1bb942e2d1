"""Write the oracle's CASCI energies f(T) for every tuple of the Hubbard-16
and synthetic M = 40 expansions to ``tests/golden/``.

This script calls only ``oracle/`` (the CPU oracle) and ``workloads/`` (the
seeded input generators); no stored value comes from the HIP path.  Each
file holds f(()) = E_ref and f(T) for every tuple T of expansion orbitals of
orders 1..k in lexicographic order (the constituent CASCI calculations of
Eq. 1), and, for reference, the increments' order sums E^(n) and the total
that the oracle's Eq. 2 recursion gives from them.

Usage: ``python tests/golden/make_mbe_goldens.py [hubbard16|synthetic40 ...]
[--workers N]``.  The oracle takes about 3 minutes (Hubbard-16) and 25
minutes (synthetic M = 40) on 8 cores.
"""
from __future__ import annotations

import argparse
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import mbe  # noqa: E402

NAMES = ("hubbard16", "synthetic40")


def fingerprint(p):
    """Sums and norms of the integrals: a check that the generator still makes
    the same inputs (to rounding; bitwise equality across BLAS builds is not
    expected)."""
    return (float(np.sum(p.h1)), float(np.sum(p.eri)), float(np.linalg.norm(p.h1)),
            float(np.linalg.norm(p.eri)))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def write(name, workers):
    p = W.problem(name)
    t0 = time.time()
    r = mbe.mbe(p, workers=workers)
    wall = time.time() - t0
    path = os.path.join(HERE, f"mbe_{name}.txt")
    fp = fingerprint(p)
    with open(path, "w") as f:
        f.write(f"# Oracle CASCI energies f(T) of every tuple of the {name} expansion\n")
        f.write("# (the constituent CASCI calculations of Eq. 1; increments by Eq. 2).\n")
        f.write("# Written by tests/golden/make_mbe_goldens.py from oracle/ and workloads/ only.\n")
        f.write(f"# problem {name}: M={p.norb} occ={p.occ} ref={p.ref} exp={p.exp} "
                f"max_order={p.max_order}\n")
        f.write("# fingerprint " + " ".join(f"{x:.17g}" for x in fp) + "\n")
        f.write(f"# oracle wall {wall:.1f} s on {workers} worker processes, {cpu_model()}\n")
        f.write(f"# e_ref {r['e_ref']:.17g}\n")
        f.write("# e_order " + " ".join(f"{x:.17g}" for x in r["e_order"]) + "\n")
        f.write(f"# e_total {r['e_total']:.17g}\n")
        f.write("# lines: expansion orbitals of T (comma separated, '-' for the empty "
                "tuple) and f(T) in E_h\n")
        f.write(f"- {r['e_ref']:.17g}\n")
        for t, ft in zip(r["tuples"], r["f"]):
            f.write(",".join(str(x) for x in t) + f" {ft:.17g}\n")
    print(f"{name}: {len(r['tuples']) + 1} CASCIs in {wall:.1f} s -> {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(NAMES))
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for n in a.names:
        if n not in NAMES:
            raise SystemExit(f"unknown workload {n}")
        write(n, a.workers)


if __name__ == "__main__":
    main()
