"""Seeded synthetic graph generators (symmetric CSR), shared input source of
the CPU oracle and the GPU library.  Holds no label-propagation arithmetic.

Graphs come back as :class:`CSR` with numpy arrays ``row_ptr`` (uint64, n+1),
``col`` (uint32, m, ascending inside each row, no self-loops, no duplicates,
both directions of every edge) and ``w`` (uint32 or None).  Every generator is
a pure function of its arguments (counter-based RNG), independent of the
number of OpenMP threads.

The shapes stand in for the paper's SuiteSparse classes (Table 1): R-MAT for
the skewed web and social graphs, a damaged lattice with shortcuts for the
road networks (mean degree about 2-3), and planted-partition SBMs.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (-O3, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "graphgen.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _GG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64),
                ("row_ptr", ctypes.POINTER(ctypes.c_uint64)),
                ("col", ctypes.POINTER(ctypes.c_uint32)),
                ("w", ctypes.POINTER(ctypes.c_uint32))]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_GG)
        u32, u64, dbl, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        lib.gg_rmat.argtypes = [u32, u32, dbl, dbl, dbl, u64, i32, P]
        lib.gg_road.argtypes = [u32, u32, dbl, dbl, u32, u32, u64, P]
        lib.gg_sbm.argtypes = [u32, u32, dbl, dbl, u64, P]
        lib.gg_from_edges.argtypes = [u32, u64, ctypes.c_void_p, ctypes.c_void_p, P]
        lib.gg_weights.argtypes = [P, u64, u32, u32]
        lib.gg_sbm_batch.argtypes = [u32, u32, u32, dbl, dbl, u64, P, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_sbm_batch.restype = ctypes.c_int
        lib.gg_free.argtypes = [P]
        lib.gg_version.restype = u32
        lib.gg_hash.argtypes = [u64, u64, u64]
        lib.gg_hash.restype = u64
        for f in (lib.gg_rmat, lib.gg_road, lib.gg_sbm, lib.gg_from_edges, lib.gg_weights):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray | None = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) if len(self.row_ptr) else 0

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col).tobytes())
        if self.w is not None:
            h.update(np.ascontiguousarray(self.w).tobytes())
        return h.hexdigest()[:16]


def _take(g: _GG, name: str) -> CSR:
    lib = _load()
    n, m = int(g.n), int(g.m)
    rp = np.ctypeslib.as_array(g.row_ptr, shape=(n + 1,)).copy()
    col = (np.ctypeslib.as_array(g.col, shape=(m,)).copy() if m else np.zeros(0, np.uint32))
    w = None
    if g.w:
        w = np.ctypeslib.as_array(g.w, shape=(m,)).copy() if m else np.zeros(0, np.uint32)
    lib.gg_free(ctypes.byref(g))
    return CSR(n=n, row_ptr=rp, col=col, w=w, name=name)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen {what} failed with code {rc}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 22, permute: bool = True) -> CSR:
    """Plain R-MAT (no per-level noise), edge_factor * 2^scale samples, a
    seeded vertex permutation, then self-loops dropped, symmetrised and
    deduplicated; unit weights (w=None)."""
    g = _GG()
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, seed, int(permute), ctypes.byref(g)), "rmat")
    return _take(g, f"rmat{scale}_ef{edge_factor}_s{seed}")


def road(rows: int = 4096, cols: int = 4096, p_delete: float = 0.3, p_diag: float = 0.01,
         wmin: int = 1, wmax: int = 8, seed: int = 4096) -> CSR:
    """Lattice rows x cols, each lattice edge deleted with p_delete, each
    vertex off the last row adds a diagonal to the next row with p_diag;
    integer weights uniform in [wmin, wmax] (wmax=0: unweighted)."""
    g = _GG()
    _check(_load().gg_road(rows, cols, p_delete, p_diag, wmin, wmax, seed, ctypes.byref(g)), "road")
    return _take(g, f"road{rows}x{cols}_s{seed}")


def sbm(n: int = 10000, k: int = 100, p_in: float = 0.1, p_out: float = 0.001, seed: int = 1) -> CSR:
    """Planted partition with k contiguous near-equal blocks (planted label of
    v is its block); unit weights."""
    g = _GG()
    _check(_load().gg_sbm(n, k, p_in, p_out, seed, ctypes.byref(g)), "sbm")
    return _take(g, f"sbm{n}_k{k}_s{seed}")


def sbm_blocks(n: int, k: int) -> np.ndarray:
    """Planted block of every vertex for :func:`sbm` (first n%k blocks larger)."""
    q, r = divmod(n, k)
    sizes = np.array([q + 1] * r + [q] * (k - r), dtype=np.int64)
    return np.repeat(np.arange(k, dtype=np.uint32), sizes)


def from_edges(n: int, edges, weights: tuple[int, int, int] | None = None) -> CSR:
    """Symmetric deduplicated CSR from an undirected edge list (self-loops
    dropped).  ``weights=(seed, lo, hi)`` attaches pair-hashed weights."""
    e = np.asarray(list(edges), dtype=np.uint32).reshape(-1, 2)
    eu = np.ascontiguousarray(e[:, 0])
    ev = np.ascontiguousarray(e[:, 1])
    g = _GG()
    lib = _load()
    _check(lib.gg_from_edges(n, len(e), eu.ctypes.data if len(e) else None,
                             ev.ctypes.data if len(e) else None, ctypes.byref(g)), "from_edges")
    if weights is not None:
        _check(lib.gg_weights(ctypes.byref(g), *weights), "weights")
    return _take(g, f"edges{n}")


def from_csr_arrays(n: int, row_ptr, col, w=None, name: str = "") -> CSR:
    """Wrap caller-built CSR arrays without any check (error-path tests)."""
    return CSR(n=n, row_ptr=np.asarray(row_ptr, dtype=np.uint64), col=np.asarray(col, dtype=np.uint32),
               w=None if w is None else np.asarray(w, dtype=np.uint32), name=name)


def with_weights(g: CSR, seed: int, lo: int, hi: int) -> CSR:
    """Copy of g with pair-hashed integer weights uniform in [lo, hi]."""
    gg = _GG()
    lib = _load()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    gg.n = g.n
    gg.m = g.m
    gg.row_ptr = rp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    gg.col = col.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    gg.w = None
    # gg_weights only reads row_ptr/col and allocates w
    _check(lib.gg_weights(ctypes.byref(gg), seed, lo, hi), "weights")
    w = np.ctypeslib.as_array(gg.w, shape=(g.m,)).copy() if g.m else np.zeros(0, np.uint32)
    # free only the weight array that the library allocated
    libc = ctypes.CDLL(None)
    libc.free.argtypes = [ctypes.c_void_p]
    libc.free(ctypes.cast(gg.w, ctypes.c_void_p))
    return CSR(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w, name=g.name + f"_w{lo}-{hi}")


def hash64(seed: int, stream: int, ctr: int) -> int:
    """The generator's counter-based draw (exposed for tests)."""
    return int(_load().gg_hash(seed, stream, ctr))


def version() -> int:
    return int(_load().gg_version())


@dataclass
class Batch:
    """G graphs packed in one CSR: graph g owns vertices gv[g]..gv[g+1]."""
    csr: CSR
    gv: np.ndarray          # uint64, G+1
    k: np.ndarray           # uint32, G: planted block count per graph

    @property
    def G(self) -> int:
        return len(self.gv) - 1

    def graph(self, g: int) -> CSR:
        """Graph g alone, with local vertex ids."""
        v0, v1 = int(self.gv[g]), int(self.gv[g + 1])
        rp = self.csr.row_ptr[v0:v1 + 1]
        a0, a1 = int(rp[0]), int(rp[-1])
        col = (self.csr.col[a0:a1].astype(np.int64) - v0).astype(np.uint32)
        w = None if self.csr.w is None else self.csr.w[a0:a1].copy()
        return CSR(n=v1 - v0, row_ptr=(rp - rp[0]).astype(np.uint64), col=col, w=w, name=f"{self.csr.name}[{g}]")


def sbm_batch(G: int = 4096, n_min: int = 200, n_max: int = 200000, deg_in: float = 12.0,
              deg_out: float = 2.0, seed: int = 4096) -> Batch:
    """G planted-partition graphs with n log-uniform in [n_min, n_max], 8..64
    blocks (each >= 25 vertices), expected intra/inter degrees deg_in and
    deg_out, packed into one CSR (unit weights)."""
    g = _GG()
    gv = np.zeros(G + 1, dtype=np.uint64)
    kk = np.zeros(G, dtype=np.uint32)
    _check(_load().gg_sbm_batch(G, n_min, n_max, deg_in, deg_out, seed, ctypes.byref(g),
                                gv.ctypes.data, kk.ctypes.data), "sbm_batch")
    return Batch(_take(g, f"sbmbatch{G}_{n_min}-{n_max}_s{seed}"), gv, kk)


def pack(graphs) -> Batch:
    """Pack CSR graphs (local ids) into one CSR; graph g gets the vertex
    range gv[g]..gv[g+1]-1.  Weights are kept if every graph has them."""
    graphs = list(graphs)
    gv = np.zeros(len(graphs) + 1, dtype=np.uint64)
    for i, g in enumerate(graphs):
        gv[i + 1] = gv[i] + g.n
    rps, cols, ws, base_arc = [np.zeros(1, np.uint64)], [], [], 0
    weighted = bool(graphs) and all(g.w is not None for g in graphs)
    for i, g in enumerate(graphs):
        rps.append((g.row_ptr[1:].astype(np.uint64) + np.uint64(base_arc)))
        cols.append((g.col.astype(np.int64) + int(gv[i])).astype(np.uint32))
        if weighted:
            ws.append(g.w.astype(np.uint32))
        base_arc += g.m
    rp = np.concatenate(rps)
    col = np.concatenate(cols) if cols else np.zeros(0, np.uint32)
    w = (np.concatenate(ws) if ws else np.zeros(0, np.uint32)) if weighted else None
    k = np.zeros(len(graphs), dtype=np.uint32)
    return Batch(CSR(n=int(gv[-1]), row_ptr=rp, col=col, w=w, name=f"pack{len(graphs)}"), gv, k)
