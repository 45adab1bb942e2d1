"""ctypes declarations of the C ABI in ``include/mbefci.h``.

Loads ``libmbefci.so`` from this package directory.  There is no fallback:
if the library is missing the import of the binding raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbefci.so")

OK, EINVAL, ENOMEM, ENOTCONV, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BATCHED, PER_LAUNCH = 0, 1

ERROR_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ENOTCONV: "ENOTCONV", EDEVICE: "EDEVICE",
               EUNSUPPORTED: "EUNSUPPORTED"}

# every symbol include/mbefci.h declares
EXPORTS = (
    "mbefci_default_opts", "mbefci_create", "mbefci_destroy", "mbefci_last_error",
    "mbefci_set_opts", "mbefci_set_allocator", "mbefci_num_strings", "mbefci_num_links",
    "mbefci_strings", "mbefci_link_table", "mbefci_strings_device", "mbefci_link_table_device",
    "mbefci_num_tuples", "mbefci_hdiag", "mbefci_sigma", "mbefci_sigma_noalloc", "mbefci_casci",
    "mbefci_casci_batch", "mbefci_casci_rdm", "mbefci_sym_ndet", "mbefci_casci_sym",
    "mbefci_sigma_sym", "mbefci_mbe_forward", "mbefci_mbe_backward",
    "mbefci_mbe_screened", "mbefci_screened_tuples", "mbefci_partition", "mbefci_time_kernels",
    "mbefci_probe_peaks",
)


# workspace allocator callbacks: alloc(bytes, user) -> device pointer or NULL,
# release(ptr, user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Opts(ctypes.Structure):
    _fields_ = [
        ("conv_tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("max_space", ctypes.c_int32),
        ("nguess", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("keep_ci", ctypes.c_int32),
        ("validate", ctypes.c_int32),
        ("sigma_pass_mb", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("pspace", ctypes.c_int32),
        ("screen_batch", ctypes.c_int32),
        ("max_workspace", ctypes.c_int64),
        ("tune_cache", ctypes.c_char_p),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("norb", ctypes.c_int32),
        ("h1", ctypes.c_void_p),
        ("eri", ctypes.c_void_p),
        ("e_const", ctypes.c_double),
        ("nocc", ctypes.c_int32),
        ("occ", ctypes.POINTER(ctypes.c_int32)),
        ("nref", ctypes.c_int32),
        ("ref", ctypes.POINTER(ctypes.c_int32)),
        ("nexp", ctypes.c_int32),
        ("exp", ctypes.POINTER(ctypes.c_int32)),
        ("max_order", ctypes.c_int32),
        ("orbsym", ctypes.POINTER(ctypes.c_int32)),
    ]


class Screen(ctypes.Structure):
    _fields_ = [
        ("t_init", ctypes.c_double),
        ("a", ctypes.c_double),
        ("m_init", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("ntuples", ctypes.c_int64),
        ("nsingle", ctypes.c_int64),
        ("sigma_calls", ctypes.c_int64),
        ("ndet_total", ctypes.c_int64),
        ("max_iters", ctypes.c_int32),
        ("first_failed", ctypes.c_int32),
        ("nbuckets", ctypes.c_int32),
        ("graph_launches", ctypes.c_int32),
        ("ms_total", ctypes.c_double),
        ("ms_solve", ctypes.c_double),
        ("ms_tune", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 64),
        ("launches", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("ms_per_launch", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
        ("ndet", ctypes.c_double),
    ]

    def as_dict(self):
        return {"name": self.name.decode(), "launches": self.launches,
                "ms_per_launch": self.ms_per_launch, "flops": self.flops, "bytes": self.bytes,
                "ndet": self.ndet}


_lib = None


def load():
    """Load and declare the library (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is not built; run `python -m paper_1910_03527_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pvp = ctypes.POINTER(ctypes.c_void_p)
    L.mbefci_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.mbefci_default_opts.restype = None
    L.mbefci_create.argtypes = [ctypes.c_int, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.mbefci_create.restype = ctypes.c_int
    L.mbefci_destroy.argtypes = [vp]
    L.mbefci_destroy.restype = None
    L.mbefci_last_error.argtypes = [vp]
    L.mbefci_last_error.restype = ctypes.c_char_p
    L.mbefci_set_opts.argtypes = [vp, ctypes.POINTER(Opts)]
    L.mbefci_set_opts.restype = ctypes.c_int
    L.mbefci_set_allocator.argtypes = [vp, ALLOC_FN, RELEASE_FN, vp]
    L.mbefci_set_allocator.restype = ctypes.c_int
    L.mbefci_num_strings.argtypes = [i32, i32]
    L.mbefci_num_strings.restype = i64
    L.mbefci_num_links.argtypes = [i32, i32]
    L.mbefci_num_links.restype = i32
    L.mbefci_num_tuples.argtypes = [i32, i32]
    L.mbefci_num_tuples.restype = i64
    L.mbefci_strings.argtypes = [i32, i32, vp]
    L.mbefci_strings.restype = ctypes.c_int
    L.mbefci_link_table.argtypes = [i32, i32, vp]
    L.mbefci_link_table.restype = ctypes.c_int
    L.mbefci_strings_device.argtypes = [vp, i32, i32, vp, vp]
    L.mbefci_strings_device.restype = ctypes.c_int
    L.mbefci_link_table_device.argtypes = [vp, i32, i32, vp, vp]
    L.mbefci_link_table_device.restype = ctypes.c_int
    L.mbefci_hdiag.argtypes = [vp, i32, i32, i32, vp, vp, dbl, vp, vp]
    L.mbefci_hdiag.restype = ctypes.c_int
    L.mbefci_sigma.argtypes = [vp, i32, i32, i32, vp, vp, dbl, vp, vp, vp]
    L.mbefci_sigma.restype = ctypes.c_int
    L.mbefci_sigma_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, dbl, vp, vp, vp]
    L.mbefci_sigma_noalloc.restype = ctypes.c_int
    L.mbefci_casci_batch.argtypes = [vp, i32, i32, i32, i32, pvp, pvp, ctypes.POINTER(dbl),
                               ctypes.POINTER(dbl), pvp, ctypes.POINTER(Stats), vp]
    L.mbefci_casci_batch.restype = ctypes.c_int
    L.mbefci_casci.argtypes = [vp, i32, i32, i32, vp, vp, dbl, ctypes.POINTER(dbl), vp, vp, vp, vp]
    L.mbefci_casci.restype = ctypes.c_int
    pi32 = ctypes.POINTER(i32)
    L.mbefci_sym_ndet.argtypes = [i32, i32, i32, pi32, i32]
    L.mbefci_sym_ndet.restype = ctypes.c_int64
    L.mbefci_casci_sym.argtypes = [vp, i32, i32, i32, i32, pi32, i32, pvp, pvp,
                                   ctypes.POINTER(dbl), ctypes.POINTER(dbl), pvp,
                                   ctypes.POINTER(Stats), vp]
    L.mbefci_casci_sym.restype = ctypes.c_int
    L.mbefci_sigma_sym.argtypes = [vp, i32, i32, i32, pi32, i32, vp, vp, dbl, vp, vp, vp]
    L.mbefci_sigma_sym.restype = ctypes.c_int
    L.mbefci_casci_rdm.argtypes = [vp, pvp, pvp, vp]
    L.mbefci_casci_rdm.restype = ctypes.c_int
    L.mbefci_mbe_forward.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(Stats), vp]
    L.mbefci_mbe_forward.restype = ctypes.c_int
    L.mbefci_mbe_backward.argtypes = [vp, ctypes.POINTER(dbl), vp, vp, vp]
    L.mbefci_mbe_backward.restype = ctypes.c_int
    L.mbefci_mbe_screened.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(Screen),
                                      ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                      ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                      ctypes.POINTER(Stats), vp]
    L.mbefci_mbe_screened.restype = ctypes.c_int
    L.mbefci_screened_tuples.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.mbefci_screened_tuples.restype = i64
    pi32 = ctypes.POINTER(i32)
    L.mbefci_partition.argtypes = [i32, i32, i32, pi32, pi32, pi32, pi32, pi32]
    L.mbefci_partition.restype = ctypes.c_int
    L.mbefci_time_kernels.argtypes = [vp, i32, ctypes.POINTER(KernelTime), i32,
                                      ctypes.POINTER(i32)]
    L.mbefci_time_kernels.restype = ctypes.c_int
    L.mbefci_probe_peaks.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    L.mbefci_probe_peaks.restype = ctypes.c_int
    _lib = L
    return L


class MbefciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
