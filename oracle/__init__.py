"""CPU oracle for RAK label propagation, modularity and NMI.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and the two share no code.

Paper: Sahu, arXiv 2301.09125.  RAK/LPA, weighted (Section 3.2): unique
initial labels, each vertex adopts the label with the most interconnecting
weight, stop when at most a `tolerance` fraction of vertices changed
(Sections 3.2 and 4).  Modularity (Section 1) and NMI (Section 2) are the
quality measures the paper names.

Readings where the paper is silent (shared with the C source): synchronous
rounds, lowest-label tie-break for the strict mode, the paper's per-vertex
self-loop modelled by `self_weight` added to the vertex's own label, stop
after round t iff changed_t <= floor(tol * n), iteration cap `max_iter`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_libs = {}


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc -O2, sequential) and, from the same source,
    liboracle_omp.so (gcc -O2 -fopenmp: a round's vertices shared among
    threads, the paper's OpenMP form of RAK, Section 3.2)."""
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", *extra, "-shared", "-fPIC", "-std=c11", "-o", tmp,
                                   os.path.join(_HERE, "oracle.c"), "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def threads(parallel: bool = True) -> int:
    """Threads a round of the (parallel) oracle uses."""
    return int(_load(parallel).orc_threads())


def _load(parallel: bool = False):
    lib = _libs.get(parallel)
    if lib is None:
        path = _OMP_PATH if parallel else _LIB_PATH
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        vp, u32, u64, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        lib.orc_rak.argtypes = [u32, vp, vp, vp, u32, dbl, u32, vp, vp, vp, vp, vp]
        lib.orc_rak.restype = ctypes.c_int
        lib.orc_rak_round.argtypes = [u32, vp, vp, vp, u32, vp, vp, vp]
        lib.orc_rak_round.restype = ctypes.c_int64
        lib.orc_rak_round_top2.argtypes = [u32, vp, vp, vp, u32, vp, vp, vp, vp]
        lib.orc_rak_round_top2.restype = ctypes.c_int64
        lib.orc_rak_masked.argtypes = [u32, vp, vp, vp, u32, u32, vp, vp, vp, vp]
        lib.orc_rak_masked.restype = ctypes.c_int
        lib.orc_modularity.argtypes = [u32, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_modularity.restype = ctypes.c_int
        lib.orc_rak_ext.argtypes = [u32, vp, vp, vp, u32, dbl, u32, vp, ctypes.c_int, ctypes.c_int, u64, vp, vp,
                                    vp, vp, vp]
        lib.orc_rak_ext.restype = ctypes.c_int
        lib.orc_splitmix64_at.argtypes = [u64, u64]
        lib.orc_splitmix64_at.restype = u64
        lib.orc_lowbias32.argtypes = [u32]
        lib.orc_lowbias32.restype = u32
        lib.orc_half_of.argtypes = [u64, u32, u32]
        lib.orc_half_of.restype = ctypes.c_int
        lib.orc_tie_key.argtypes = [u64, u32, u32]
        lib.orc_tie_key.restype = u32
        lib.orc_copra.argtypes = [u32, vp, vp, vp, u32, ctypes.c_int, ctypes.c_int, u64, dbl, u32, vp, vp, vp, vp,
                                  vp, vp, vp]
        lib.orc_copra.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        _libs[parallel] = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({-1: "invalid input", -2: "weighted degree overflows 32 bits",
                          -3: "out of memory"}.get(code, f"error {code}"))
        self.code = code


def _arrs(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.uint32)
    return rp, col, w


def _p(a):
    return None if a is None else a.ctypes.data


@dataclass
class RakResult:
    labels: np.ndarray
    iterations: int
    converged: bool
    changed: list = field(default_factory=list)


def rak(g, tol: float = 0.05, max_iter: int = 20, self_weight: int = 1,
        init_labels: np.ndarray | None = None, parallel: bool = False) -> RakResult:
    """Synchronous RAK (Section 3.2) with the lowest-label tie-break
    (parallel: the OpenMP build of the same source)."""
    rp, col, w = _arrs(g)
    out = np.empty(g.n, dtype=np.uint32)
    ch = np.zeros(max(max_iter, 1), dtype=np.uint64)
    it = ctypes.c_uint32(0)
    cv = ctypes.c_int32(0)
    init = None if init_labels is None else np.ascontiguousarray(init_labels, dtype=np.uint32)
    rc = _load(parallel).orc_rak(g.n, rp.ctypes.data, col.ctypes.data, _p(w), self_weight, float(tol), max_iter,
                         _p(init), out.ctypes.data, ch.ctypes.data, ctypes.byref(it), ctypes.byref(cv))
    if rc:
        raise OracleError(rc)
    return RakResult(out, int(it.value), bool(cv.value), [int(x) for x in ch[: it.value]])


def rak_ext(g, tol: float = 0.05, max_iter: int = 20, self_weight: int = 1, order: str = "sync",
            tie: str = "lowest", seed: int = 0, halves: np.ndarray | None = None,
            init_labels: np.ndarray | None = None, parallel: bool = False) -> RakResult:
    """RAK (Section 3.2) with a choice of update order -- "sync" (round t
    reads round t-1) or "semisync" (two half-rounds per round over the
    vertices of each half, drawn from `seed` every round, or the split
    `halves` in every round) -- and of
    tie-break -- "lowest" (strict) or "hash" (non-strict, reproducible from
    `seed`)."""
    if order not in ("sync", "semisync") or tie not in ("lowest", "hash"):
        raise ValueError("order: sync|semisync, tie: lowest|hash")
    rp, col, w = _arrs(g)
    out = np.empty(g.n, dtype=np.uint32)
    ch = np.zeros(max(max_iter, 1), dtype=np.uint64)
    it = ctypes.c_uint32(0)
    cv = ctypes.c_int32(0)
    init = None if init_labels is None else np.ascontiguousarray(init_labels, dtype=np.uint32)
    hv = None if halves is None else np.ascontiguousarray(halves, dtype=np.uint8)
    rc = _load(parallel).orc_rak_ext(g.n, rp.ctypes.data, col.ctypes.data, _p(w), self_weight, float(tol),
                                     max_iter, _p(init), 1 if order == "semisync" else 0, 1 if tie == "hash" else 0,
                                     int(seed) & ((1 << 64) - 1), _p(hv), out.ctypes.data, ch.ctypes.data,
                                     ctypes.byref(it), ctypes.byref(cv))
    if rc:
        raise OracleError(rc)
    return RakResult(out, int(it.value), bool(cv.value), [int(x) for x in ch[: it.value]])


def splitmix64_at(seed: int, c: int) -> int:
    """Output number c+1 of SplitMix64 started from state `seed`."""
    return int(_load().orc_splitmix64_at(seed & ((1 << 64) - 1), c & ((1 << 64) - 1)))


def lowbias32(x: int) -> int:
    return int(_load().orc_lowbias32(x & 0xFFFFFFFF))


def half_of(seed: int, t: int, v: int) -> int:
    """Half (0/1) of vertex v in round t of a semi-synchronous run."""
    return int(_load().orc_half_of(seed & ((1 << 64) - 1), t, v))


def tie_key(seed: int, t: int, v: int) -> int:
    """Tie key of vertex v in round t (non-strict votes)."""
    return int(_load().orc_tie_key(seed & ((1 << 64) - 1), t, v))


def rak_round(g, labels: np.ndarray, self_weight: int = 1, active: np.ndarray | None = None,
              parallel: bool = False):
    """One synchronous round from `labels`; returns (new_labels, changed)."""
    rp, col, w = _arrs(g)
    old = np.ascontiguousarray(labels, dtype=np.uint32)
    new = np.empty_like(old)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    ch = _load(parallel).orc_rak_round(g.n, rp.ctypes.data, col.ctypes.data, _p(w), self_weight,
                               old.ctypes.data, new.ctypes.data, _p(act))
    if ch < 0:
        raise OracleError(int(ch))
    return new, int(ch)


def rak_round_top2(g, labels: np.ndarray, self_weight: int = 1):
    """One synchronous round over every vertex; returns (new_labels, changed,
    top1, top2): the winning tally of each vertex and the largest tally of
    any other label in its closed neighbourhood (0 if none)."""
    rp, col, w = _arrs(g)
    old = np.ascontiguousarray(labels, dtype=np.uint32)
    new = np.empty_like(old)
    t1 = np.zeros(g.n, dtype=np.uint64)
    t2 = np.zeros(g.n, dtype=np.uint64)
    ch = _load().orc_rak_round_top2(g.n, rp.ctypes.data, col.ctypes.data, _p(w), self_weight,
                                    old.ctypes.data, new.ctypes.data, t1.ctypes.data, t2.ctypes.data)
    if ch < 0:
        raise OracleError(int(ch))
    return new, int(ch), t1, t2


def rak_masked(g, masks: np.ndarray, self_weight: int = 1, init_labels=None):
    """Replay rounds restricted to masks[t] (uint8 [rounds, n])."""
    rp, col, w = _arrs(g)
    masks = np.ascontiguousarray(masks, dtype=np.uint8)
    rounds = masks.shape[0] if masks.ndim == 2 else 0
    out = np.empty(g.n, dtype=np.uint32)
    ch = np.zeros(max(rounds, 1), dtype=np.uint64)
    init = None if init_labels is None else np.ascontiguousarray(init_labels, dtype=np.uint32)
    rc = _load().orc_rak_masked(g.n, rp.ctypes.data, col.ctypes.data, _p(w), self_weight, rounds,
                                masks.ctypes.data, _p(init), out.ctypes.data, ch.ctypes.data)
    if rc:
        raise OracleError(rc)
    return out, [int(x) for x in ch[:rounds]]


COPRA_ONE = 1 << 16  # belonging coefficient 1 in the oracle's fixed point


@dataclass
class CopraResult:
    labels: np.ndarray      # best label of every vertex
    iterations: int
    converged: bool
    changed: list
    state: list             # per vertex: sorted [(label, coefficient * 2^16), ...] (None when raw)
    state_arrays: tuple = None  # raw: (labels [n, V], coefficients [n, V], counts [n]), uint32


def copra(g, max_labels: int = 4, tol: float = 0.01, max_iter: int = 20, order: str = "sync", tie: str = "lowest",
          seed: int = 0, raw: bool = False) -> CopraResult:
    """COPRA (Section 3.3) with fixed-point belonging coefficients, in
    synchronous or semi-synchronous rounds; the best label's ties go to the
    lowest label or, with tie="hash", to the highest priority as in rak_ext.
    See the C source for the readings taken."""
    if order not in ("sync", "semisync") or tie not in ("lowest", "hash"):
        raise ValueError("order: sync|semisync, tie: lowest|hash")
    rp, col, w = _arrs(g)
    V = int(max_labels)
    best = np.empty(g.n, dtype=np.uint32)
    sl = np.zeros(max(g.n * V, 1), dtype=np.uint32)
    sc = np.zeros(max(g.n * V, 1), dtype=np.uint32)
    sn = np.zeros(max(g.n, 1), dtype=np.uint32)
    ch = np.zeros(max(max_iter, 1), dtype=np.uint64)
    it = ctypes.c_uint32(0)
    cv = ctypes.c_int32(0)
    rc = _load().orc_copra(g.n, rp.ctypes.data, col.ctypes.data, _p(w), V, 1 if order == "semisync" else 0,
                           1 if tie == "hash" else 0,
                           int(seed) & ((1 << 64) - 1), float(tol), max_iter, best.ctypes.data,
                           sl.ctypes.data, sc.ctypes.data, sn.ctypes.data, ch.ctypes.data, ctypes.byref(it),
                           ctypes.byref(cv))
    if rc:
        raise OracleError(rc)
    changed = [int(x) for x in ch[: it.value]]
    if raw:
        return CopraResult(best, int(it.value), bool(cv.value), changed, None,
                           (sl[: g.n * V].reshape(g.n, V), sc[: g.n * V].reshape(g.n, V), sn[: g.n]))
    state = [sorted(zip(sl[v * V:v * V + sn[v]].tolist(), sc[v * V:v * V + sn[v]].tolist())) for v in range(g.n)]
    return CopraResult(best, int(it.value), bool(cv.value), changed, state)


@dataclass
class ModResult:
    q: float
    two_m: int
    sigma_in: int
    sum_k2: int


def modularity(g, labels: np.ndarray) -> ModResult:
    """Weighted Newman-Girvan modularity (Section 1), exact integer sums."""
    rp, col, w = _arrs(g)
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    q = ctypes.c_double(0)
    tm = ctypes.c_uint64(0)
    si = ctypes.c_uint64(0)
    sk = (ctypes.c_uint64 * 2)()
    rc = _load().orc_modularity(g.n, rp.ctypes.data, col.ctypes.data, _p(w), lab.ctypes.data,
                                ctypes.byref(q), ctypes.byref(tm), ctypes.byref(si), sk)
    if rc:
        raise OracleError(rc)
    return ModResult(q.value, tm.value, si.value, int(sk[0]) + (int(sk[1]) << 64))


def nmi(a, b) -> float:
    """Normalised mutual information of two partitions (Section 2 names the
    measure): 2 I(A;B) / (H(A) + H(B)), natural logarithm; 1 when both
    entropies are 0 (both partitions a single block)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    if a.size != b.size:
        raise ValueError("partitions differ in size")
    N = a.size
    if N == 0:
        return 1.0
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    pa = np.bincount(ai).astype(np.float64) / N
    pb = np.bincount(bi).astype(np.float64) / N
    joint = ai.astype(np.int64) * (int(bi.max()) + 1) + bi
    _, nij = np.unique(joint, return_counts=True)
    ja = _ // (int(bi.max()) + 1)
    jb = _ % (int(bi.max()) + 1)
    pij = nij.astype(np.float64) / N
    ha = -np.sum(pa * np.log(pa))
    hb = -np.sum(pb * np.log(pb))
    mi = np.sum(pij * (np.log(pij) - np.log(pa[ja]) - np.log(pb[jb])))
    if ha + hb == 0.0:
        return 1.0
    return float(2.0 * mi / (ha + hb))
