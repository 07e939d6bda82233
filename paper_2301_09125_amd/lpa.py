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
LPA_ETOOLARGE = -7
LPA_NOALLOC_MAX_N = 1 << 22
LPA_ORDER_SYNC, LPA_ORDER_SEMISYNC = 0, 1
LPA_TIE_LOWEST, LPA_TIE_HASH = 0, 1

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
                ("modularity", ctypes.c_uint32), ("frontier", ctypes.c_uint32),
                ("barrier_timeout_us", ctypes.c_uint32), ("order", ctypes.c_uint32), ("tie", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("reuse_csr", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("converged", ctypes.c_int32),
                ("changed_last", ctypes.c_uint64), ("arcs_processed", ctypes.c_uint64),
                ("ms_total", ctypes.c_double), ("ms_rounds", ctypes.c_double), ("ms_prepare", ctypes.c_double),
                ("modularity", ctypes.c_double), ("mod_terms", ctypes.c_uint64 * 4),
                ("changed_per_iter", ctypes.POINTER(ctypes.c_uint64)),
                ("ms_per_iter", ctypes.POINTER(ctypes.c_float)), ("cap", ctypes.c_uint32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_uint32), ("rounds", ctypes.c_uint32), ("converged_graphs", ctypes.c_uint32),
                ("arcs_processed", ctypes.c_uint64), ("ms_total", ctypes.c_double), ("ms_device", ctypes.c_double),
                ("iterations", ctypes.c_void_p), ("converged", ctypes.c_void_p), ("changed_last", ctypes.c_void_p),
                ("changed_hist", ctypes.c_void_p), ("hist_cap", ctypes.c_uint32)]


_F32 = ctypes.c_float


class _Mlp(ctypes.Structure):
    _fields_ = [("w1", (_F32 * 32) * 6), ("b1", _F32 * 32), ("w2", (_F32 * 32) * 32), ("b2", _F32 * 32),
                ("w3", _F32 * 32), ("b3", _F32), ("tau", _F32)]


class _LearnedStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("converged", ctypes.c_int32),
                ("learned_rounds", ctypes.c_uint32), ("check_round", ctypes.c_uint32),
                ("changed_last", ctypes.c_uint64), ("arcs_processed", ctypes.c_uint64),
                ("ms_total", ctypes.c_double), ("ms_rounds", ctypes.c_double),
                ("modularity", ctypes.c_double), ("mod_terms", ctypes.c_uint64 * 4),
                ("changed_per_iter", ctypes.c_void_p), ("voted_per_iter", ctypes.c_void_p),
                ("candidates_per_iter", ctypes.c_void_p), ("cap", ctypes.c_uint32)]


class _TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", _F32), ("pos_weight", _F32),
                ("seed", ctypes.c_uint64), ("val_X", ctypes.c_void_p), ("val_y", ctypes.c_void_p),
                ("val_n", ctypes.c_uint64), ("recall", _F32)]


MLP_FIELDS = ("w1", "b1", "w2", "b2", "w3", "b3")


def _mlp_to_c(model: dict) -> _Mlp:
    m = _Mlp()
    flat = np.concatenate([np.asarray(model[k], dtype=np.float32).ravel() for k in MLP_FIELDS])
    assert flat.size == 1313, flat.size
    ctypes.memmove(ctypes.addressof(m), flat.ctypes.data, flat.nbytes)
    m.tau = float(model.get("tau", 0.5))
    return m


def _mlp_from_c(m: _Mlp) -> dict:
    flat = np.frombuffer(ctypes.string_at(ctypes.addressof(m), 1313 * 4), dtype=np.float32).copy()
    out, o = {}, 0
    for k, shape in (("w1", (6, 32)), ("b1", (32,)), ("w2", (32, 32)), ("b2", (32,)), ("w3", (32,)), ("b3", ())):
        size = int(np.prod(shape)) if shape else 1
        out[k] = flat[o:o + size].reshape(shape) if shape else np.float32(flat[o])
        o += size
    out["tau"] = float(m.tau)
    return out


class _KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_uint64), ("arcs", ctypes.c_uint64)]


EXPORTS = ("lpa_default_options", "lpa_init", "lpa_run", "lpa_run_resume", "lpa_run_batch", "lpa_run_learned",
           "lpa_trace", "lpa_train", "lpa_mlp_forward", "lpa_mlp_grad", "lpa_autotune", "lpa_modularity",
           "lpa_modularity_noalloc", "lpa_run_copra",
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
    u64 = ctypes.c_uint64
    lib.lpa_run_learned.argtypes = [vp, ctypes.POINTER(_Csr), ctypes.POINTER(_Mlp), vp, dbl, u32,
                                    ctypes.POINTER(_LearnedStats), vp, u32]
    lib.lpa_trace.argtypes = [vp, ctypes.POINTER(_Csr), dbl, u32, vp, vp, u64, ctypes.POINTER(u64)]
    lib.lpa_train.argtypes = [vp, vp, vp, u64, ctypes.POINTER(_TrainOpts), ctypes.POINTER(_Mlp), vp]
    lib.lpa_mlp_forward.argtypes = [vp, ctypes.POINTER(_Mlp), vp, u64, vp]
    lib.lpa_mlp_grad.argtypes = [vp, ctypes.POINTER(_Mlp), vp, vp, u64, _F32, vp, ctypes.POINTER(_F32)]
    lib.lpa_autotune.argtypes = [vp, ctypes.POINTER(_Csr), vp, u32, u32, ctypes.POINTER(_Options),
                                 ctypes.POINTER(u32)]
    lib.lpa_modularity.argtypes = [vp, ctypes.POINTER(_Csr), vp, ctypes.POINTER(dbl),
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.lpa_modularity_noalloc.argtypes = [vp, ctypes.POINTER(_Csr), vp, ctypes.POINTER(dbl),
                                           ctypes.POINTER(ctypes.c_uint64)]
    lib.lpa_run_copra.argtypes = [vp, ctypes.POINTER(_Csr), u32, vp, vp, vp, vp, dbl, u32, ctypes.POINTER(_Stats)]
    lib.lpa_profile_get.argtypes = [vp, ctypes.POINTER(_KProf), u32, ctypes.POINTER(u32)]
    lib.lpa_profile_reset.argtypes = [vp]
    lib.lpa_destroy.argtypes = [vp]
    lib.lpa_destroy.restype = None
    lib.lpa_strerror.argtypes = [ctypes.c_int]
    lib.lpa_strerror.restype = ctypes.c_char_p
    for f in (lib.lpa_run_learned, lib.lpa_trace, lib.lpa_train, lib.lpa_mlp_forward, lib.lpa_mlp_grad,
              lib.lpa_autotune):
        f.restype = ctypes.c_int
    for f in (lib.lpa_init, lib.lpa_run, lib.lpa_run_resume, lib.lpa_run_batch, lib.lpa_modularity, lib.lpa_modularity_noalloc,
              lib.lpa_run_copra, lib.lpa_profile_get,
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
    ms_prepare: float = 0.0


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


@dataclass
class LearnedStats:
    iterations: int
    converged: bool
    learned_rounds: int
    check_round: int
    changed_last: int
    arcs_processed: int
    ms_total: float
    ms_rounds: float
    changed: list
    voted: list
    candidates: list
    modularity: float = 0.0
    mod_terms: dict = field(default_factory=dict)


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
                     {"two_m": int(t[0]), "sigma_in": int(t[1]), "sum_k2": int(t[2]) + (int(t[3]) << 64)},
                     st.ms_prepare)

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

    def run_copra(self, g: DeviceGraph, max_labels: int = 4, tol: float = 0.01, max_iter: int = 20,
                  state: bool = False, labels_out=None):
        """COPRA (lpa_run_copra); returns (best labels int32 tensor viewed as
        u32, Stats) or, with state, (best, Stats, (labels [n, V], coefs
        [n, V], count [n]) int32 tensors)."""
        import torch
        dev = g.row_ptr.device
        if labels_out is None:
            labels_out = torch.empty(g.n, dtype=torch.int32, device=dev)
        V = int(max_labels)
        sl = sc = sn = None
        if state:
            sl = torch.zeros((g.n, V), dtype=torch.int32, device=dev)
            sc = torch.zeros((g.n, V), dtype=torch.int32, device=dev)
            sn = torch.zeros(g.n, dtype=torch.int32, device=dev)
        st, ch, ms = self._stats(max_iter)
        c = g._c()
        p = (lambda t: t.data_ptr() if (t is not None and g.n) else None)
        rc = _load().lpa_run_copra(self._h, ctypes.byref(c), V, p(labels_out), p(sl), p(sc), p(sn), float(tol),
                                   int(max_iter), ctypes.byref(st))
        if rc:
            raise LpaError(rc, "lpa_run_copra")
        out = (labels_out, self._pack(st, ch, ms))
        return out + ((sl, sc, sn),) if state else out

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

    def run_learned(self, g: DeviceGraph, model: dict, tol: float = 0.05, max_iter: int = 20, labels_out=None,
                    masks: bool = False):
        """RAK with the learned frontier; returns (labels, LearnedStats, masks
        (u8 tensor [rounds, n] by original id) or None)."""
        import torch
        if labels_out is None:
            labels_out = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        mk = torch.zeros((max_iter, g.n), dtype=torch.uint8, device=g.row_ptr.device) if masks else None
        cap = max(max_iter, 1)
        ch, vo, ca = (np.zeros(cap, np.uint64) for _ in range(3))
        st = _LearnedStats()
        st.changed_per_iter, st.voted_per_iter, st.candidates_per_iter = ch.ctypes.data, vo.ctypes.data, ca.ctypes.data
        st.cap = cap
        m = _mlp_to_c(model)
        c = g._c()
        rc = _load().lpa_run_learned(self._h, ctypes.byref(c), ctypes.byref(m), labels_out.data_ptr() if g.n else None,
                                     float(tol), int(max_iter), ctypes.byref(st),
                                     mk.data_ptr() if (mk is not None and g.n) else None, max_iter if masks else 0)
        if rc:
            raise LpaError(rc, "lpa_run_learned")
        k = st.iterations
        stats = LearnedStats(k, bool(st.converged), st.learned_rounds, st.check_round, st.changed_last,
                             st.arcs_processed, st.ms_total, st.ms_rounds, [int(x) for x in ch[:k]],
                             [int(x) for x in vo[:k]], [int(x) for x in ca[:k]], st.modularity,
                             {"two_m": int(st.mod_terms[0]), "sigma_in": int(st.mod_terms[1]),
                              "sum_k2": int(st.mod_terms[2]) | (int(st.mod_terms[3]) << 64)})
        return labels_out, stats, (mk[:k] if mk is not None else None)

    def trace(self, g: DeviceGraph, tol: float = 0.05, max_iter: int = 20, cap: int | None = None):
        """Training samples of a plain run: (X float32 [count, 6], y uint8 [count]) on the device."""
        import torch
        if cap is None:
            cap = g.n * max(max_iter - 1, 0)
        X = torch.empty((max(cap, 1), 6), dtype=torch.float32, device=g.row_ptr.device)
        y = torch.empty(max(cap, 1), dtype=torch.uint8, device=g.row_ptr.device)
        cnt = ctypes.c_uint64(0)
        c = g._c()
        rc = _load().lpa_trace(self._h, ctypes.byref(c), float(tol), int(max_iter), X.data_ptr(), y.data_ptr(),
                               cap, ctypes.byref(cnt))
        if rc:
            raise LpaError(rc, "lpa_trace")
        if cnt.value > cap:
            raise RuntimeError(f"trace holds {cnt.value} samples, more than cap={cap}")
        return X[:cnt.value], y[:cnt.value]

    def train(self, X, y, model: dict, epochs: int = 3, batch: int = 65536, lr: float = 3e-3,
              pos_weight: float = 1.0, seed: int = 1, val=None, recall: float = 0.99):
        """Train on device samples; returns (model dict with tau set from the
        validation samples when given, loss per epoch)."""
        m = _mlp_to_c(model)
        o = _TrainOpts()
        o.epochs, o.batch, o.lr, o.pos_weight, o.seed = epochs, batch, lr, pos_weight, seed
        if val is not None:
            o.val_X, o.val_y, o.val_n, o.recall = val[0].data_ptr(), val[1].data_ptr(), val[0].shape[0], recall
        losses = np.zeros(max(epochs, 1), np.float32)
        rc = _load().lpa_train(self._h, X.data_ptr(), y.data_ptr(), X.shape[0], ctypes.byref(o), ctypes.byref(m),
                               losses.ctypes.data)
        if rc:
            raise LpaError(rc, "lpa_train")
        return _mlp_from_c(m), [float(x) for x in losses[:epochs]]

    def mlp_forward(self, model: dict, X):
        """Logits of device samples X (float32 [N, 6]) with the inference arithmetic."""
        import torch
        z = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        m = _mlp_to_c(model)
        rc = _load().lpa_mlp_forward(self._h, ctypes.byref(m), X.data_ptr(), X.shape[0], z.data_ptr())
        if rc:
            raise LpaError(rc, "lpa_mlp_forward")
        return z

    def mlp_grad(self, model: dict, X, y, pos_weight: float = 1.0):
        """(loss, gradient dict) of the training loss over all samples."""
        m = _mlp_to_c(model)
        g = np.zeros(1313, np.float32)
        loss = ctypes.c_float(0)
        rc = _load().lpa_mlp_grad(self._h, ctypes.byref(m), X.data_ptr(), y.data_ptr(), X.shape[0],
                                  float(pos_weight), g.ctypes.data, ctypes.byref(loss))
        if rc:
            raise LpaError(rc, "lpa_mlp_grad")
        out = _Mlp()
        ctypes.memmove(ctypes.addressof(out), g.ctypes.data, g.nbytes)
        d = _mlp_from_c(out)
        d.pop("tau")
        return float(loss.value), d

    def autotune(self, g: DeviceGraph, graph_vptr=None, rounds: int = 2):
        """Pick the fastest degree-bin thresholds for g (batched when
        graph_vptr is given); returns (options dict, candidates timed)."""
        o = _Options()
        n = ctypes.c_uint32(0)
        gv = None if graph_vptr is None else np.ascontiguousarray(np.asarray(graph_vptr, dtype=np.uint64))
        c = g._c()
        rc = _load().lpa_autotune(self._h, ctypes.byref(c), gv.ctypes.data if gv is not None else None,
                                  0 if gv is None else len(gv) - 1, rounds, ctypes.byref(o), ctypes.byref(n))
        if rc:
            raise LpaError(rc, "lpa_autotune")
        self.options = {k: getattr(o, k) for k, _ in _Options._fields_}
        return dict(self.options), int(n.value)

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

    def modularity_noalloc(self, g: DeviceGraph, labels):
        """As modularity(), through lpa_modularity_noalloc (fixed scratch,
        no allocation; n <= LPA_NOALLOC_MAX_N)."""
        q = ctypes.c_double(0)
        terms = (ctypes.c_uint64 * 4)()
        c = g._c()
        rc = _load().lpa_modularity_noalloc(self._h, ctypes.byref(c), labels.data_ptr() if g.n else None,
                                            ctypes.byref(q), terms)
        if rc:
            raise LpaError(rc, "lpa_modularity_noalloc")
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
