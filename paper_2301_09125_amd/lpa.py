"""Python binding of liblpa.so (include/lpa.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the label
propagation runs in the library's HIP kernels.  There is no fallback: if the
library cannot be loaded, or no GPU is present, calls raise.

Method: RAK label propagation (arXiv 2301.09125, Section 3.2) with
synchronous rounds and the lowest-label tie-break; modularity (Section 1).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpa.so")

LPA_OK, LPA_EINVAL, LPA_EOVERFLOW, LPA_ENOMEM, LPA_EDEVICE, LPA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LPA_ETIMEDOUT = -6

_lib = None


class LpaError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _load().lpa_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("self_weight", ctypes.c_uint32), ("thread_max", ctypes.c_uint32),
                ("group_max", ctypes.c_uint32), ("wave_max", ctypes.c_uint32),
                ("wide_max", ctypes.c_uint32), ("merge_max", ctypes.c_uint32), ("profile", ctypes.c_uint32),
                ("modularity", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("converged", ctypes.c_int32),
                ("changed_last", ctypes.c_uint64), ("arcs_processed", ctypes.c_uint64),
                ("ms_total", ctypes.c_double), ("ms_rounds", ctypes.c_double),
                ("modularity", ctypes.c_double), ("mod_terms", ctypes.c_uint64 * 4),
                ("changed_per_iter", ctypes.POINTER(ctypes.c_uint64)),
                ("ms_per_iter", ctypes.POINTER(ctypes.c_float)), ("cap", ctypes.c_uint32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_uint32), ("rounds", ctypes.c_uint32), ("converged_graphs", ctypes.c_uint32),
                ("arcs_processed", ctypes.c_uint64), ("ms_total", ctypes.c_double), ("ms_device", ctypes.c_double),
                ("iterations", ctypes.c_void_p), ("converged", ctypes.c_void_p), ("changed_last", ctypes.c_void_p),
                ("changed_hist", ctypes.c_void_p), ("hist_cap", ctypes.c_uint32)]


class _KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_uint64), ("arcs", ctypes.c_uint64)]


EXPORTS = ("lpa_default_options", "lpa_init", "lpa_run", "lpa_run_resume", "lpa_run_batch", "lpa_modularity",
           "lpa_profile_get", "lpa_profile_reset", "lpa_destroy", "lpa_strerror")


def _load():
    """Load liblpa.so (building it only if nothing is built yet)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_double
    lib.lpa_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.lpa_default_options.restype = None
    lib.lpa_init.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(_Options)]
    lib.lpa_run.argtypes = [vp, ctypes.POINTER(_Csr), vp, dbl, u32, ctypes.POINTER(_Stats)]
    lib.lpa_run_resume.argtypes = [vp, ctypes.POINTER(_Csr), vp, dbl, u32, ctypes.POINTER(_Stats)]
    lib.lpa_run_batch.argtypes = [vp, ctypes.POINTER(_Csr), vp, u32, vp, dbl, u32, ctypes.POINTER(_BatchStats)]
    lib.lpa_modularity.argtypes = [vp, ctypes.POINTER(_Csr), vp, ctypes.POINTER(dbl),
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.lpa_profile_get.argtypes = [vp, ctypes.POINTER(_KProf), u32, ctypes.POINTER(u32)]
    lib.lpa_profile_reset.argtypes = [vp]
    lib.lpa_destroy.argtypes = [vp]
    lib.lpa_destroy.restype = None
    lib.lpa_strerror.argtypes = [ctypes.c_int]
    lib.lpa_strerror.restype = ctypes.c_char_p
    for f in (lib.lpa_init, lib.lpa_run, lib.lpa_run_resume, lib.lpa_run_batch, lib.lpa_modularity, lib.lpa_profile_get,
              lib.lpa_profile_reset):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def library():
    return _load()


def default_options() -> dict:
    o = _Options()
    _load().lpa_default_options(ctypes.byref(o))
    return {k: getattr(o, k) for k, _ in _Options._fields_}


class DeviceGraph:
    """A CSR resident in device memory (torch tensors hold the storage).

    row_ptr: int64 tensor viewed as u64[n+1]; col: int32 tensor viewed as
    u32[m]; w: int32 tensor viewed as u32[m] or None (unit weights)."""

    def __init__(self, n: int, row_ptr, col, w=None, name: str = ""):
        self.n = int(n)
        self.row_ptr = row_ptr
        self.col = col
        self.w = w
        self.name = name

    @property
    def m(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_csr(cls, g, device="cuda", weights: bool = True) -> "DeviceGraph":
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.uint64).view(np.int64)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.uint32).view(np.int32)).to(device)
        w = None
        if weights and g.w is not None:
            w = torch.from_numpy(np.ascontiguousarray(g.w, dtype=np.uint32).view(np.int32)).to(device)
        return cls(g.n, rp, col, w, getattr(g, "name", ""))

    def _c(self) -> _Csr:
        c = _Csr()
        c.n = self.n
        c.m = self.m
        c.row_ptr = self.row_ptr.data_ptr()
        c.col = self.col.data_ptr() if self.m else None
        c.w = None if self.w is None else self.w.data_ptr()
        return c

    def nbytes(self) -> int:
        return 8 * (self.n + 1) + 4 * self.m + (0 if self.w is None else 4 * self.m)


@dataclass
class Stats:
    iterations: int
    converged: bool
    changed_last: int
    arcs_processed: int
    ms_total: float
    ms_rounds: float
    changed: list = field(default_factory=list)
    ms_per_iter: list = field(default_factory=list)
    modularity: float = 0.0
    mod_terms: dict = field(default_factory=dict)


@dataclass
class BatchStats:
    graphs: int
    rounds: int
    converged_graphs: int
    arcs_processed: int
    ms_total: float
    ms_device: float
    iterations: np.ndarray      # u32[G]
    converged: np.ndarray       # bool[G]
    changed_last: np.ndarray    # u64[G]
    changed_hist: np.ndarray    # u64[G, hist_cap]

    def changed(self, g: int) -> list:
        """Changed counts of graph g's rounds (up to hist_cap of them)."""
        k = min(int(self.iterations[g]), self.changed_hist.shape[1])
        return [int(x) for x in self.changed_hist[g, :k]]


class Context:
    """One lpa_ctx bound to a device and a HIP stream (torch's current stream
    by default)."""

    def __init__(self, device: int = 0, stream=None, **options):
        import torch
        lib = _load()
        if not torch.cuda.is_available():
            raise RuntimeError("liblpa needs a ROCm GPU; none is visible")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        o = _Options()
        lib.lpa_default_options(ctypes.byref(o))
        for k, v in options.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, int(v))
        h = ctypes.c_void_p()
        rc = lib.lpa_init(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(o))
        if rc:
            raise LpaError(rc, "lpa_init")
        self._h = h
        self.options = {k: getattr(o, k) for k, _ in _Options._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _load().lpa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _stats(self, cap: int):
        st = _Stats()
        ch = (ctypes.c_uint64 * max(cap, 1))()
        ms = (ctypes.c_float * max(cap, 1))()
        st.changed_per_iter = ctypes.cast(ch, ctypes.POINTER(ctypes.c_uint64))
        st.ms_per_iter = ctypes.cast(ms, ctypes.POINTER(ctypes.c_float))
        st.cap = cap
        return st, ch, ms

    @staticmethod
    def _pack(st, ch, ms) -> Stats:
        k = st.iterations
        t = st.mod_terms
        return Stats(st.iterations, bool(st.converged), st.changed_last, st.arcs_processed, st.ms_total,
                     st.ms_rounds, [int(x) for x in ch[:k]], [float(x) for x in ms[:k]], st.modularity,
                     {"two_m": int(t[0]), "sigma_in": int(t[1]), "sum_k2": int(t[2]) + (int(t[3]) << 64)})

    def run(self, g: DeviceGraph, tol: float = 0.05, max_iter: int = 20, labels_out=None):
        """RAK from L0(v) = v; returns (labels int32 tensor viewed as u32, Stats)."""
        import torch
        if labels_out is None:
            labels_out = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        st, ch, ms = self._stats(max_iter)
        c = g._c()
        rc = _load().lpa_run(self._h, ctypes.byref(c), labels_out.data_ptr() if g.n else None, float(tol),
                             int(max_iter), ctypes.byref(st))
        if rc:
            raise LpaError(rc, "lpa_run")
        return labels_out, self._pack(st, ch, ms)

    def run_resume(self, g: DeviceGraph, labels, tol: float = 0.05, max_iter: int = 20):
        """RAK from the labels in `labels` (updated in place)."""
        st, ch, ms = self._stats(max_iter)
        c = g._c()
        rc = _load().lpa_run_resume(self._h, ctypes.byref(c), labels.data_ptr() if g.n else None,
                                    float(tol), int(max_iter), ctypes.byref(st))
        if rc:
            raise LpaError(rc, "lpa_run_resume")
        return labels, self._pack(st, ch, ms)

    def run_batch(self, g: DeviceGraph, graph_vptr, tol: float = 0.05, max_iter: int = 20, labels_out=None,
                  hist_cap: int | None = None):
        """RAK on the graphs packed in g (graph k owns vertices graph_vptr[k] ..
        graph_vptr[k+1]-1); labels come back as ids local to each graph."""
        import torch
        gv = np.ascontiguousarray(np.asarray(graph_vptr, dtype=np.uint64))
        G = max(len(gv) - 1, 0)
        if labels_out is None:
            labels_out = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        cap = max_iter if hist_cap is None else hist_cap
        it = np.zeros(max(G, 1), np.uint32)
        cv = np.zeros(max(G, 1), np.int32)
        last = np.zeros(max(G, 1), np.uint64)
        hist = np.zeros((max(G, 1), max(cap, 1)), np.uint64)
        st = _BatchStats()
        st.iterations, st.converged, st.changed_last = it.ctypes.data, cv.ctypes.data, last.ctypes.data
        st.changed_hist, st.hist_cap = hist.ctypes.data, cap
        c = g._c()
        rc = _load().lpa_run_batch(self._h, ctypes.byref(c), gv.ctypes.data if len(gv) else None, G,
                                   labels_out.data_ptr() if g.n else None, float(tol), int(max_iter),
                                   ctypes.byref(st))
        if rc:
            raise LpaError(rc, "lpa_run_batch")
        return labels_out, BatchStats(st.graphs, st.rounds, st.converged_graphs, st.arcs_processed, st.ms_total,
                                      st.ms_device, it[:G], cv[:G].astype(bool), last[:G], hist[:G, :cap])

    def modularity(self, g: DeviceGraph, labels):
        """(Q, {'two_m', 'sigma_in', 'sum_k2'}) computed on the device."""
        q = ctypes.c_double(0)
        terms = (ctypes.c_uint64 * 4)()
        c = g._c()
        rc = _load().lpa_modularity(self._h, ctypes.byref(c), labels.data_ptr() if g.n else None,
                                    ctypes.byref(q), terms)
        if rc:
            raise LpaError(rc, "lpa_modularity")
        return q.value, {"two_m": int(terms[0]), "sigma_in": int(terms[1]),
                         "sum_k2": int(terms[2]) + (int(terms[3]) << 64)}

    def profile(self) -> list:
        recs = (_KProf * 16)()
        cnt = ctypes.c_uint32(0)
        rc = _load().lpa_profile_get(self._h, recs, 16, ctypes.byref(cnt))
        if rc:
            raise LpaError(rc, "lpa_profile_get")
        return [{"name": recs[i].name.decode(), "launches": recs[i].launches, "ms": recs[i].ms,
                 "bytes": recs[i].bytes, "arcs": recs[i].arcs} for i in range(min(cnt.value, 16))]

    def profile_reset(self):
        rc = _load().lpa_profile_reset(self._h)
        if rc:
            raise LpaError(rc, "lpa_profile_reset")


def labels_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
