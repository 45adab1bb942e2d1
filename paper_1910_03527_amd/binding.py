"""Argument marshalling between torch tensors and the C ABI (``_lib``)."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import BATCHED, PER_LAUNCH, MbefciError  # noqa: F401

TYPE1, TYPE2, TYPE3 = 1, 2, 3   # reference/expansion partitions (mbefci_partition)


def num_strings(norb: int, nelec: int) -> int:
    return int(_lib.load().mbefci_num_strings(norb, nelec))


def num_links(norb: int, nelec: int) -> int:
    return int(_lib.load().mbefci_num_links(norb, nelec))


def num_tuples(nexp: int, max_order: int) -> int:
    return int(_lib.load().mbefci_num_tuples(nexp, max_order))


def strings(norb: int, nelec: int) -> np.ndarray:
    """The string bitmasks of nelec electrons in norb orbitals, ascending
    (mbefci_strings: host, no context, no device)."""
    n = num_strings(norb, nelec)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    rc = _lib.load().mbefci_strings(norb, nelec, out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise MbefciError(rc, "mbefci_strings failed")
    return out[:n]


def link_table(norb: int, nelec: int) -> np.ndarray:
    """[nstr, nlink, 4] = (p, q, J, sign) single-excitation links
    (mbefci_link_table: host, no context, no device)."""
    n, nl = num_strings(norb, nelec), num_links(norb, nelec)
    out = np.zeros((max(n, 1), max(nl, 1), 4), dtype=np.int32)
    rc = _lib.load().mbefci_link_table(norb, nelec, out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise MbefciError(rc, "mbefci_link_table failed")
    return out[:n, :nl]


def sym_ndet(norb: int, nalpha: int, nbeta: int, orbsym, wfnsym: int = 0) -> int:
    """Determinants of irrep ``wfnsym`` (mbefci_sym_ndet: host, no context)."""
    nd = int(_lib.load().mbefci_sym_ndet(norb, nalpha, nbeta, _i32(orbsym), int(wfnsym)))
    if nd < 0:
        raise MbefciError(nd, "mbefci_sym_ndet failed")
    return nd


def _dev_f64(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape) and t.numel() != math.prod(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _i32(xs):
    xs = [int(x) for x in xs]
    arr = (ctypes.c_int32 * max(1, len(xs)))(*xs)
    return arr


def partition(kind: int, norb: int, occ):
    """(ref, exp) of the paper's Type-1/2/3 partition (mbefci_partition)."""
    L = _lib.load()
    occ_a = _i32(occ)
    ref = (ctypes.c_int32 * norb)()
    exp = (ctypes.c_int32 * norb)()
    nr, nx = ctypes.c_int32(), ctypes.c_int32()
    rc = L.mbefci_partition(int(kind), int(norb), len(occ), occ_a, ref, ctypes.byref(nr), exp,
                            ctypes.byref(nx))
    if rc != 0:
        raise MbefciError(rc, "mbefci_partition failed")
    return list(ref)[:nr.value], list(exp)[:nx.value]


class Context:
    """One library context on one device (mbefci_create)."""

    def __init__(self, device: int = 0, **opts):
        self._L = _lib.load()
        self.device = int(device)
        o = _lib.Opts()
        self._L.mbefci_default_opts(ctypes.byref(o))
        self._cache = None
        for k, v in opts.items():
            if k == "tune_cache":
                self._cache = None if v is None else str(v).encode()
                v = self._cache
            setattr(o, k, v)
        self._opts = o
        h = ctypes.c_void_p()
        rc = self._L.mbefci_create(self.device, ctypes.byref(o), ctypes.byref(h))
        if rc != 0:
            raise MbefciError(rc, "mbefci_create failed")
        self._h = h
        self.last_stats = None
        self._fwd = None

    # ------------------------------------------------------------ plumbing
    def close(self):
        if getattr(self, "_h", None):
            self._L.mbefci_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc):
        if rc != 0:
            msg = self._L.mbefci_last_error(self._h)
            raise MbefciError(rc, msg.decode() if msg else "")

    @property
    def opts(self) -> dict:
        return {k: getattr(self._opts, k) for k, _ in _lib.Opts._fields_}

    def set_opts(self, **opts):
        o = _lib.Opts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(self._opts), ctypes.sizeof(o))
        for k, v in opts.items():
            if k == "tune_cache":
                self._cache = None if v is None else str(v).encode()
                v = self._cache
            setattr(o, k, v)
        self._check(self._L.mbefci_set_opts(self._h, ctypes.byref(o)))
        self._opts = o

    def use_torch_allocator(self, enable: bool = True):
        """Take the context's workspaces from torch's caching allocator
        (mbefci_set_allocator), or give them back to hipMalloc."""
        if enable:
            dev = self.device

            def alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
                except RuntimeError:
                    return None

            def release(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            cbs = (_lib.ALLOC_FN(alloc), _lib.RELEASE_FN(release))
        else:
            cbs = (_lib.ALLOC_FN(), _lib.RELEASE_FN())
        self._check(self._L.mbefci_set_allocator(self._h, cbs[0], cbs[1], None))
        self._fwd = None
        self._allocator = cbs  # the callbacks must outlive every arena they made

    def _dev(self):
        return torch.device("cuda", self.device)

    # ------------------------------------------------------ integer layer
    def strings(self, norb: int, nelec: int) -> torch.Tensor:
        n = num_strings(norb, nelec)
        out = torch.empty(max(n, 1), dtype=torch.int64, device=self._dev())
        self._check(self._L.mbefci_strings_device(self._h, norb, nelec,
                                                  ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out[:n]

    def link_table(self, norb: int, nelec: int) -> torch.Tensor:
        n, L = num_strings(norb, nelec), num_links(norb, nelec)
        out = torch.empty((max(n, 1), max(L, 1), 4), dtype=torch.int32, device=self._dev())
        self._check(self._L.mbefci_link_table_device(self._h, norb, nelec,
                                                     ctypes.c_void_p(out.data_ptr()),
                                                     self._stream()))
        return out[:n, :L]

    # --------------------------------------------------- one Hamiltonian
    def hdiag(self, h1, eri, nalpha: int, nbeta: int, e_core: float = 0.0) -> torch.Tensor:
        n = h1.shape[0]
        _dev_f64(h1, (n, n), "h1")
        _dev_f64(eri, (n, n, n, n), "eri")
        nd = num_strings(n, nalpha) * num_strings(n, nbeta)
        out = torch.empty(nd, dtype=torch.float64, device=self._dev())
        self._check(self._L.mbefci_hdiag(self._h, n, nalpha, nbeta, ctypes.c_void_p(h1.data_ptr()),
                                         ctypes.c_void_p(eri.data_ptr()), float(e_core),
                                         ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def sigma(self, h1, eri, nalpha: int, nbeta: int, c, e_core: float = 0.0) -> torch.Tensor:
        n = h1.shape[0]
        _dev_f64(h1, (n, n), "h1")
        _dev_f64(eri, (n, n, n, n), "eri")
        nd = num_strings(n, nalpha) * num_strings(n, nbeta)
        _dev_f64(c, (nd,), "c")
        out = torch.empty(nd, dtype=torch.float64, device=self._dev())
        self._check(self._L.mbefci_sigma(self._h, n, nalpha, nbeta, ctypes.c_void_p(h1.data_ptr()),
                                         ctypes.c_void_p(eri.data_ptr()), float(e_core),
                                         ctypes.c_void_p(c.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def sigma_noalloc(self, h1, eri, nalpha: int, nbeta: int, c, out, e_core: float = 0.0):
        """sigma = H c into the caller's ``out`` through mbefci_sigma_noalloc
        (no device allocation: the library's static scratch array); returns
        ``out``."""
        n = h1.shape[0]
        _dev_f64(h1, (n, n), "h1")
        _dev_f64(eri, (n, n, n, n), "eri")
        nd = num_strings(n, nalpha) * num_strings(n, nbeta)
        _dev_f64(c, (nd,), "c")
        _dev_f64(out, (nd,), "out")
        self._check(self._L.mbefci_sigma_noalloc(
            self._h, n, nalpha, nbeta, ctypes.c_void_p(h1.data_ptr()),
            ctypes.c_void_p(eri.data_ptr()), float(e_core), ctypes.c_void_p(c.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    # --------------------------------------------------------- CASCI batch
    def casci(self, h1s, eris, nalpha: int, nbeta: int, e_core=None, want_ci: bool = False):
        """Lowest eigenvalues (host list) of a batch of same-shape CASCIs;
        with ``want_ci`` also their CI vectors (device tensors [Na*Nb])."""
        if isinstance(h1s, torch.Tensor) and h1s.dim() == 2:
            h1s, eris = [h1s], [eris]
        nprob = len(h1s)
        n = h1s[0].shape[0]
        for i in range(nprob):
            _dev_f64(h1s[i], (n, n), f"h1[{i}]")
            _dev_f64(eris[i], (n, n, n, n), f"eri[{i}]")
        ecore = [0.0] * nprob if e_core is None else [float(x) for x in e_core]
        nd = num_strings(n, nalpha) * num_strings(n, nbeta)
        hp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in h1s])
        gp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in eris])
        ec = (ctypes.c_double * nprob)(*ecore)
        eo = (ctypes.c_double * nprob)()
        cis = None
        cp = None
        if want_ci:
            cis = [torch.empty(nd, dtype=torch.float64, device=self._dev()) for _ in range(nprob)]
            cp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in cis])
        st = _lib.Stats()
        self._check(self._L.mbefci_casci_batch(self._h, nprob, n, nalpha, nbeta,
                                         ctypes.cast(hp, ctypes.POINTER(ctypes.c_void_p)),
                                         ctypes.cast(gp, ctypes.POINTER(ctypes.c_void_p)), ec, eo,
                                         None if cp is None else
                                         ctypes.cast(cp, ctypes.POINTER(ctypes.c_void_p)),
                                         ctypes.byref(st), self._stream()))
        self.last_stats = st.as_dict()
        self._casci_shape = (nprob, n)
        e = list(eo)
        return (e, cis) if want_ci else e

    def casci_one(self, h1, eri, nalpha: int, nbeta: int, e_core: float = 0.0,
                  want_ci: bool = False, want_rdm: bool = False):
        """One CASCI through mbefci_casci: the energy, and on request the CI
        vector [Na*Nb] and (gamma [n, n], Gamma [n, n, n, n]) as device
        tensors: returns a dict with keys e, ci, rdm1, rdm2."""
        n = h1.shape[0]
        _dev_f64(h1, (n, n), "h1")
        _dev_f64(eri, (n, n, n, n), "eri")
        nd = num_strings(n, nalpha) * num_strings(n, nbeta)
        ci = torch.empty(nd, dtype=torch.float64, device=self._dev()) if want_ci else None
        g1 = torch.empty((n, n), dtype=torch.float64, device=self._dev()) if want_rdm else None
        g2 = torch.empty((n,) * 4, dtype=torch.float64, device=self._dev()) if want_rdm else None
        e = ctypes.c_double()

        def p(t):
            return None if t is None else ctypes.c_void_p(t.data_ptr())

        self._check(self._L.mbefci_casci(self._h, n, nalpha, nbeta, p(h1), p(eri), float(e_core),
                                         ctypes.byref(e), p(ci), p(g1), p(g2), self._stream()))
        self._casci_shape = (1, n)
        return {"e": e.value, "ci": ci, "rdm1": g1, "rdm2": g2}

    def casci_rdm(self, want_rdm2: bool = True):
        """(gamma [nprob, n, n], Gamma [nprob, n, n, n, n]) of the last casci."""
        nprob, n = self._casci_shape
        g1 = torch.empty((nprob, n, n), dtype=torch.float64, device=self._dev())
        g2 = torch.empty((nprob, n, n, n, n), dtype=torch.float64, device=self._dev()) \
            if want_rdm2 else None
        p1 = (ctypes.c_void_p * nprob)(*[g1[i].data_ptr() for i in range(nprob)])
        p2 = (ctypes.c_void_p * nprob)(*[g2[i].data_ptr() for i in range(nprob)]) \
            if want_rdm2 else None
        self._check(self._L.mbefci_casci_rdm(
            self._h, ctypes.cast(p1, ctypes.POINTER(ctypes.c_void_p)),
            None if p2 is None else ctypes.cast(p2, ctypes.POINTER(ctypes.c_void_p)),
            self._stream()))
        return g1, g2

    # ---------------------------------------------------------------- MBE
    def mbe_forward(self, h1, eri, occ, ref, exp, max_order: int, e_const: float = 0.0,
                    want_increments: bool = False):
        """Returns dict(e_ref, e_order [k], e_total, increments?) (host floats)."""
        M = h1.shape[0]
        _dev_f64(h1, (M, M), "h1")
        _dev_f64(eri, (M, M, M, M), "eri")
        occ_a, ref_a, exp_a = _i32(occ), _i32(ref), _i32(exp)
        pb = _lib.Problem(M, h1.data_ptr(), eri.data_ptr(), float(e_const), len(occ), occ_a,
                          len(ref), ref_a, len(exp), exp_a, int(max_order))
        e_ref = ctypes.c_double()
        e_tot = ctypes.c_double()
        e_ord = (ctypes.c_double * max(1, max_order))()
        nt = num_tuples(len(exp), max_order)
        inc = (ctypes.c_double * max(1, nt))() if want_increments else None
        fen = (ctypes.c_double * max(1, nt))() if want_increments else None
        st = _lib.Stats()
        self._check(self._L.mbefci_mbe_forward(self._h, ctypes.byref(pb), ctypes.byref(e_ref),
                                               e_ord, ctypes.byref(e_tot), inc, fen,
                                               ctypes.byref(st), self._stream()))
        self.last_stats = st.as_dict()
        self._fwd = (M, max_order)
        out = {"e_ref": e_ref.value, "e_order": list(e_ord)[:max_order], "e_total": e_tot.value}
        if want_increments:
            out["increments"] = list(inc)[:nt]
            out["energies"] = list(fen)[:nt]
        return out

    def mbe_screened(self, h1, eri, occ, ref, exp, max_order: int, t_init: float = 1e-10,
                     m_init: int = 3, a: float = 5.0, e_const: float = 0.0,
                     want_tuples: bool = False, orbsym=None):
        """Screened order-by-order expansion (mbefci_mbe_screened).  Returns
        dict(e_ref, e_order [k], e_total, n_order [k]) and, with want_tuples,
        per_order: list over orders of (tuples int32 [n][order], increments).
        ``orbsym``: point-group irreps (0..7) of the MOs, or None; with them
        every CASCI is solved in the totally symmetric irrep on the blocked
        path."""
        M = h1.shape[0]
        _dev_f64(h1, (M, M), "h1")
        _dev_f64(eri, (M, M, M, M), "eri")
        occ_a, ref_a, exp_a = _i32(occ), _i32(ref), _i32(exp)
        sym_a = _i32(orbsym) if orbsym is not None else None
        pb = _lib.Problem(M, h1.data_ptr(), eri.data_ptr(), float(e_const), len(occ), occ_a,
                          len(ref), ref_a, len(exp), exp_a, int(max_order),
                          ctypes.cast(sym_a, ctypes.POINTER(ctypes.c_int32)) if sym_a else None)
        sc = _lib.Screen(float(t_init), float(a), int(m_init), 0)
        e_ref = ctypes.c_double()
        e_tot = ctypes.c_double()
        e_ord = (ctypes.c_double * max(1, max_order))()
        n_ord = (ctypes.c_int64 * max(1, max_order))()
        st = _lib.Stats()
        self._check(self._L.mbefci_mbe_screened(self._h, ctypes.byref(pb), ctypes.byref(sc),
                                                ctypes.byref(e_ref), e_ord, ctypes.byref(e_tot),
                                                n_ord, ctypes.byref(st), self._stream()))
        self.last_stats = st.as_dict()
        self._fwd = None
        out = {"e_ref": e_ref.value, "e_order": list(e_ord)[:max_order], "e_total": e_tot.value,
               "n_order": list(n_ord)[:max_order]}
        if want_tuples:
            per = []
            for k in range(1, max_order + 1):
                n = int(n_ord[k - 1])
                tu = (ctypes.c_int32 * max(1, n * k))()
                inc = (ctypes.c_double * max(1, n))()
                got = self._L.mbefci_screened_tuples(self._h, k, tu, inc)
                if got < 0:
                    self._check(int(got))
                arr = np.frombuffer(tu, dtype=np.int32, count=n * k).reshape(n, k).copy()
                per.append((arr, list(inc)[:n]))
            out["per_order"] = per
        return out

    # ---------------------------------------------- point-group blocked
    def casci_sym(self, h1s, eris, nalpha: int, nbeta: int, orbsym, wfnsym: int = 0,
                  e_core=None, want_ci: bool = False):
        """Lowest eigenvalues of a batch of same-shape CASCIs in irrep
        ``wfnsym`` (mbefci_casci_sym); with ``want_ci`` also the CI vectors in
        the blocked layout of include/mbefci.h."""
        if isinstance(h1s, torch.Tensor) and h1s.dim() == 2:
            h1s, eris = [h1s], [eris]
        nprob = len(h1s)
        n = h1s[0].shape[0]
        for i in range(nprob):
            _dev_f64(h1s[i], (n, n), f"h1[{i}]")
            _dev_f64(eris[i], (n, n, n, n), f"eri[{i}]")
        nd = sym_ndet(n, nalpha, nbeta, orbsym, wfnsym)
        ecore = [0.0] * nprob if e_core is None else [float(x) for x in e_core]
        hp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in h1s])
        gp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in eris])
        ec = (ctypes.c_double * nprob)(*ecore)
        eo = (ctypes.c_double * nprob)()
        cis = cp = None
        if want_ci:
            cis = [torch.empty(max(nd, 1), dtype=torch.float64, device=self._dev())
                   for _ in range(nprob)]
            cp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in cis])
        st = _lib.Stats()
        self._check(self._L.mbefci_casci_sym(
            self._h, nprob, n, nalpha, nbeta, _i32(orbsym), int(wfnsym),
            ctypes.cast(hp, ctypes.POINTER(ctypes.c_void_p)),
            ctypes.cast(gp, ctypes.POINTER(ctypes.c_void_p)), ec, eo,
            None if cp is None else ctypes.cast(cp, ctypes.POINTER(ctypes.c_void_p)),
            ctypes.byref(st), self._stream()))
        self.last_stats = st.as_dict()
        e = list(eo)
        return (e, [t[:nd] for t in cis]) if want_ci else e

    def sigma_sym(self, h1, eri, nalpha: int, nbeta: int, orbsym, wfnsym: int, c,
                  e_core: float = 0.0) -> torch.Tensor:
        """sigma = H c on the determinants of irrep ``wfnsym`` (blocked layout;
        mbefci_sigma_sym)."""
        n = h1.shape[0]
        _dev_f64(h1, (n, n), "h1")
        _dev_f64(eri, (n, n, n, n), "eri")
        nd = sym_ndet(n, nalpha, nbeta, orbsym, wfnsym)
        _dev_f64(c, (nd,), "c")
        out = torch.empty(nd, dtype=torch.float64, device=self._dev())
        self._check(self._L.mbefci_sigma_sym(
            self._h, n, nalpha, nbeta, _i32(orbsym), int(wfnsym), ctypes.c_void_p(h1.data_ptr()),
            ctypes.c_void_p(eri.data_ptr()), float(e_core), ctypes.c_void_p(c.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def time_kernels(self, reps: int = 5):
        """Per-launch device times of the sigma kernels of the last forward
        (mbefci_time_kernels): list of dicts."""
        cap = 64
        arr = (_lib.KernelTime * cap)()
        cnt = ctypes.c_int32()
        self._check(self._L.mbefci_time_kernels(self._h, int(reps), arr, cap, ctypes.byref(cnt)))
        return [arr[i].as_dict() for i in range(min(cnt.value, cap))]

    def probe_peaks(self):
        """Measured FP64 MFMA and copy peaks of the device (mbefci_probe_peaks):
        dict(fp64_mfma_tflops, copy_gbps)."""
        tf, gb = ctypes.c_double(), ctypes.c_double()
        self._check(self._L.mbefci_probe_peaks(self._h, ctypes.byref(tf), ctypes.byref(gb)))
        return {"fp64_mfma_tflops": tf.value, "copy_gbps": gb.value}

    def mbe_backward(self, grad_out):
        """d(g0 E_ref + sum_n g_n E^(n)) / d(h1, eri) of the last forward."""
        if self._fwd is None:
            raise MbefciError(_lib.EINVAL, "mbe_backward before mbe_forward")
        M, k = self._fwd
        g = [float(x) for x in grad_out]
        if len(g) != 1 + k:
            raise ValueError(f"grad_out must hold {1 + k} values")
        ga = (ctypes.c_double * len(g))(*g)
        dh = torch.empty((M, M), dtype=torch.float64, device=self._dev())
        dg = torch.empty((M, M, M, M), dtype=torch.float64, device=self._dev())
        self._check(self._L.mbefci_mbe_backward(self._h, ga, ctypes.c_void_p(dh.data_ptr()),
                                                ctypes.c_void_p(dg.data_ptr()), self._stream()))
        return dh, dg


def casci(h1, eri, nalpha: int, nbeta: int, e_core: float = 0.0, want_rdm: bool = False,
          **opts):
    """One CASCI on the device of ``h1`` (mbefci_casci):
    the lowest eigenvalue of the S_z sector (nalpha, nbeta) plus ``e_core``,
    and with ``want_rdm`` also (gamma [n, n], Gamma [n, n, n, n]) in the
    chemist convention E = sum h gamma + 1/2 sum (pq|rs) Gamma + e_core.
    ``opts`` are Context options.  A context is created and closed per call;
    batches of CASCIs go through Context.casci."""
    dev = h1.device.index if h1.device.index is not None else torch.cuda.current_device()
    ctx = Context(dev, **opts)
    try:
        r = ctx.casci_one(h1, eri, nalpha, nbeta, e_core, want_rdm=want_rdm)
        return (r["e"], r["rdm1"], r["rdm2"]) if want_rdm else r["e"]
    finally:
        ctx.close()


class MBEEnergy(torch.autograd.Function):
    """E = [E_ref, E^(1), ..., E^(k)] as a differentiable function of the MO
    integrals: ``MBEEnergy.apply(h1, eri, ctx, occ, ref, exp, max_order)``;
    E_MBE = out.sum().  The backward contracts the upstream gradient with the
    weighted CASCI RDMs (dE/dh = gamma, dE/d(pq|rs) = Gamma/2)."""

    @staticmethod
    def forward(actx, h1, eri, context, occ, ref, exp, max_order, e_const=0.0):
        r = context.mbe_forward(h1.detach(), eri.detach(), occ, ref, exp, max_order, e_const)
        actx.context = context
        return torch.tensor([r["e_ref"], *r["e_order"]], dtype=torch.float64, device=h1.device)

    @staticmethod
    def backward(actx, grad):
        g = grad.detach().to("cpu", torch.float64).tolist()
        dh, dg = actx.context.mbe_backward(g)
        return dh, dg, None, None, None, None, None, None
