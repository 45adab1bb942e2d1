"""The C-ABI library builds, loads and exports every symbol of include/mbefci.h
(no compute calls: this runs without a GPU)."""
import ctypes
import math
import os
import re

import pytest

from paper_1910_03527_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "mbefci.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"\b(mbefci_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1910_03527_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert declared == sorted(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_integer_closed_forms(lib):
    for n in range(0, 17):
        for k in range(0, n + 1):
            assert lib.mbefci_num_strings(n, k) == math.comb(n, k)
            assert lib.mbefci_num_links(n, k) == k * (n - k + 1)
    assert lib.mbefci_num_strings(3, 4) == 0
    assert lib.mbefci_num_tuples(8, 8) == 255
    assert lib.mbefci_num_tuples(10, 4) == 385
    assert lib.mbefci_num_tuples(34, 3) == 6579
    assert lib.mbefci_num_tuples(12, 6) == 2509
    assert lib.mbefci_num_tuples(5, 6) == 0


def test_default_options(lib):
    o = _lib.Opts()
    lib.mbefci_default_opts(ctypes.byref(o))
    assert o.conv_tol == 1e-6 and o.max_space == 16 and o.nguess == 2
    assert o.mode == _lib.BATCHED and o.keep_ci == 1 and o.validate == 1


def test_null_context_is_rejected(lib):
    assert lib.mbefci_mbe_forward(None, None, None, None, None, None, None, None, None) == _lib.EINVAL
    assert lib.mbefci_strings(None, 4, 2, None, None) == _lib.EINVAL
    assert lib.mbefci_last_error(None) == b"null context"


def test_struct_layouts_match_header():
    # mbefci_problem: int32, 2 pointers, double, (int32, ptr) x 3, int32
    assert ctypes.sizeof(_lib.Problem) == 4 + 4 + 8 + 8 + 8 + 3 * (8 + 8) + 8
    assert ctypes.sizeof(_lib.Stats) == 4 * 8 + 4 * 4 + 3 * 8
