"""Readers of the stored oracle values in ``tests/golden/`` (test helpers)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_mbe_golden(name):
    """(fingerprint, f_ref, {tuple: f}) from tests/golden/mbe_<name>.txt."""
    fp = None
    f_ref = None
    f = {}
    with open(os.path.join(GOLDEN, f"mbe_{name}.txt")) as fh:
        for line in fh:
            if line.startswith("# fingerprint"):
                fp = [float(x) for x in line.split()[2:]]
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split()
            if key == "-":
                f_ref = float(val)
            else:
                f[tuple(int(x) for x in key.split(","))] = float(val)
    return fp, f_ref, f


def read_large_goldens():
    """name -> oracle energy from tests/golden/casci_large.txt."""
    out = {}
    with open(os.path.join(GOLDEN, "casci_large.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = line.split()
            out[w[0]] = float(w[1])
    return out
