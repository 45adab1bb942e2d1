"""The C-ABI library builds, loads and exports every symbol of include/mbefci.h
(no compute calls: this runs without a GPU)."""
import ctypes
import math
import os
import re

import numpy as np
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
    assert o.conv_tol == 1e-6 and o.max_space == 5 and o.nguess == 1
    assert o.mode == _lib.BATCHED and o.keep_ci == 1 and o.validate == 1
    assert o.precond == 0 and o.pspace == 112


def test_null_context_is_rejected(lib):
    assert lib.mbefci_mbe_forward(None, None, None, None, None, None, None, None, None) == _lib.EINVAL
    assert lib.mbefci_strings_device(None, 4, 2, None, None) == _lib.EINVAL
    assert lib.mbefci_casci(None, 4, 2, 2, None, None, 0.0, None, None, None, None, None) == \
        _lib.EINVAL
    assert lib.mbefci_mbe_screened(None, None, None, None, None, None, None, None, None) == \
        _lib.EINVAL
    assert lib.mbefci_screened_tuples(None, 1, None, None) == _lib.EINVAL
    assert lib.mbefci_set_allocator(None, _lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == _lib.EINVAL
    assert lib.mbefci_last_error(None) == b"null context"


@pytest.mark.parametrize("n,k", [(0, 0), (1, 0), (1, 1), (4, 2), (6, 3), (7, 2), (8, 5),
                                 (10, 5), (12, 6), (14, 7), (9, 0), (9, 9)])
def test_host_integer_layer_bit_exact(lib, n, k):
    """mbefci_strings / mbefci_link_table on the host (no context, no device)
    against the oracle's tables, bit for bit."""
    from oracle import strings as ostr
    from paper_1910_03527_amd import link_table, strings
    s = strings(n, k)
    assert s.dtype == np.uint64 and np.array_equal(s, np.array(ostr.strings(n, k), dtype=np.uint64))
    if n <= 12:
        t = link_table(n, k)
        exp = np.array(ostr.link_table(n, k), dtype=np.int32).reshape(t.shape)
        assert np.array_equal(t, exp)


def test_host_integer_layer_rejects_bad_shapes(lib):
    buf = (ctypes.c_uint64 * 8)()
    assert lib.mbefci_strings(3, 4, buf) == _lib.EINVAL
    assert lib.mbefci_strings(-1, 0, buf) == _lib.EINVAL
    assert lib.mbefci_strings(4, 2, None) == _lib.EINVAL
    assert lib.mbefci_link_table(33, 2, buf) == _lib.EINVAL
    assert lib.mbefci_strings(64, 32, buf) == _lib.EINVAL  # more than 2^31 - 1 strings


def test_sym_ndet_matches_oracle_sectors(lib):
    """mbefci_sym_ndet (host, no context) against the oracle's sector sizes,
    and the paper's Cr2 CASCI size (CAS(16,16), two orbitals per D2h irrep:
    2.07e7 determinants, Fig. 3 discussion)."""
    from oracle import sym
    from paper_1910_03527_amd import sym_ndet
    for n, na, nb, osym in [(6, 3, 3, [0, 1, 2, 3, 0, 1]), (7, 3, 4, [1, 4, 4, 7, 0, 2, 3]),
                            (8, 4, 4, [0, 5, 3, 6, 0, 1, 7, 2]), (5, 0, 2, [3, 3, 1, 0, 6])]:
        dims = sym.sector_dims(n, na, nb, osym)
        assert [sym_ndet(n, na, nb, osym, g) for g in range(8)] == dims
    assert sym_ndet(16, 8, 8, [p // 2 for p in range(16)], 0) == 20708900
    bad = (ctypes.c_int32 * 4)(0, 1, 8, 0)
    assert lib.mbefci_sym_ndet(4, 2, 2, bad, 0) == _lib.EINVAL


def test_struct_layouts_match_header(tmp_path):
    """ctypes layouts equal the C compiler's layout of include/mbefci.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mbefci_opts": _lib.Opts, "mbefci_problem": _lib.Problem,
               "mbefci_stats": _lib.Stats, "mbefci_screen": _lib.Screen,
               "mbefci_kernel_time": _lib.KernelTime}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mbefci.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('  return 0;\n}')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
