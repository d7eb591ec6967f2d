"""CPU oracle for exact max-flow / min-cut (static and after capacity updates).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the product
library never does.  It shares no code with the GPU path: the arithmetic lives
in ``mf_oracle.c`` (plain, sequential C) plus the brute-force enumeration below.

Functions
---------
dinic(g)                    O1: value, canonical source side S*, valid per-edge flow
fifo_push_relabel(g)        O2: value and canonical source side (independent algorithm)
brute_force_min_cut(g)      O3: value and union of all minimum source sides (n <= 16)
PairGraph.build(g)          merged arc pairs (bi-directional CSR, Sec. 5.1)
PaperSeq                    O4: the paper's Alg. 1/2/3/4/5 run sequentially
validate(pg, cf, e, s, t)   V: state checks + phase-two completion to a valid flow
bfs_heights(pg, cf, e, s, t) exact global-relabel heights of a residual state
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class _Nullable:
    """ctypes argtype that accepts a numpy array of a fixed dtype or None."""

    def __init__(self, dtype):
        self.dtype = np.dtype(dtype)

    def from_param(self, obj):
        if obj is None:
            return None
        if not isinstance(obj, np.ndarray) or obj.dtype != self.dtype or not obj.flags.c_contiguous:
            raise TypeError(f"expected contiguous {self.dtype} array")
        return obj.ctypes.data_as(C.c_void_p)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.orc_dinic.restype = C.c_int64
        L.orc_dinic.argtypes = [C.c_int32, C.c_int64, _i64p, _i32p, _i32p, C.c_int32, C.c_int32,
                                _Nullable(np.uint8), _Nullable(np.int64)]
        L.orc_fifo_push_relabel.restype = C.c_int64
        L.orc_fifo_push_relabel.argtypes = [C.c_int32, C.c_int64, _i64p, _i32p, _i32p, C.c_int32,
                                            C.c_int32, _Nullable(np.uint8)]
        L.orc_pairs_count.restype = C.c_int64
        L.orc_pairs_count.argtypes = [C.c_int32, C.c_int64, _i64p, _i32p]
        L.orc_pairs_build.restype = C.c_int32
        L.orc_pairs_build.argtypes = [C.c_int32, C.c_int64, _i64p, _i32p, _i32p, _i32p, _i32p,
                                      _i32p, _i32p, _i32p]
        L.orc_paper_init.restype = None
        L.orc_paper_init.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p, C.c_int32,
                                     _i32p, _i64p, _i32p]
        L.orc_paper_global_relabel.restype = None
        L.orc_paper_global_relabel.argtypes = [C.c_int32, _i32p, _i32p, _i32p, _i32p, _i64p,
                                               C.c_int32, C.c_int32, _i32p]
        L.orc_paper_loop.restype = C.c_int32
        L.orc_paper_loop.argtypes = [C.c_int32, _i32p, _i32p, _i32p, _i32p, _i64p, _i32p,
                                     C.c_int32, C.c_int32, C.c_int32, C.c_int64, _i64p]
        L.orc_paper_value.restype = C.c_int64
        L.orc_paper_value.argtypes = [C.c_int32, _i64p, C.c_int32, C.c_int32]
        L.orc_paper_apply_updates.restype = C.c_int32
        L.orc_paper_apply_updates.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p,
                                              _i32p, _i32p, _i32p, _i64p, C.c_int32, _i64p, _i32p,
                                              C.c_int64]
        L.orc_validate.restype = C.c_int32
        L.orc_validate.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p, _i64p,
                                   C.c_int32, C.c_int32, _u8p, C.POINTER(C.c_int64),
                                   _Nullable(np.int64)]
        _LIB = L
    return _LIB


def _csr(g):
    return (np.ascontiguousarray(g.row_ptr, dtype=np.int64),
            np.ascontiguousarray(g.col, dtype=np.int32),
            np.ascontiguousarray(g.cap, dtype=np.int32))


def _cap_or(g, cap):
    return np.ascontiguousarray(g.cap if cap is None else cap, dtype=np.int32)


# --------------------------------------------------------------------------
# O1 / O2 / O3
# --------------------------------------------------------------------------

def dinic(g, cap=None):
    """O1.  Returns (value, side uint8[n] with 1 = canonical source side S*,
    per-edge flow int64[m])."""
    rp, col, _ = _csr(g)
    c = _cap_or(g, cap)
    side = np.zeros(g.n, dtype=np.uint8)
    flow = np.zeros(max(1, col.shape[0]), dtype=np.int64)
    v = lib().orc_dinic(g.n, col.shape[0], rp, col, c, g.s, g.t, side, flow)
    if v < 0:
        raise MemoryError("oracle allocation failed")
    return int(v), side, flow[: col.shape[0]]


def fifo_push_relabel(g, cap=None):
    """O2.  Returns (value, side)."""
    rp, col, _ = _csr(g)
    c = _cap_or(g, cap)
    side = np.zeros(g.n, dtype=np.uint8)
    v = lib().orc_fifo_push_relabel(g.n, col.shape[0], rp, col, c, g.s, g.t, side)
    if v < 0:
        raise MemoryError("oracle allocation failed")
    return int(v), side


def brute_force_min_cut(g, cap=None):
    """O3: enumerate every S with s in S, t not in S (n <= 16).  The cut
    capacity is the sum of c(u,v) over edges leaving S (Sec. 2.1 / the
    max-flow min-cut theorem).  Returns (min value, uint8 union of all
    minimising S)."""
    n, s, t = g.n, g.s, g.t
    if n > 16:
        raise ValueError("brute force is limited to n <= 16")
    c = np.asarray(g.cap if cap is None else cap, dtype=np.int64)
    tails = g.tails().astype(np.int64)
    heads = np.asarray(g.col, dtype=np.int64)
    others = [v for v in range(n) if v not in (s, t)]
    k = len(others)
    masks = np.arange(1 << k, dtype=np.int64)
    member = np.zeros((1 << k, n), dtype=bool)
    for j, v in enumerate(others):
        member[:, v] = (masks >> j) & 1
    member[:, s] = True
    member[:, t] = False
    if tails.size:
        crossing = member[:, tails] & ~member[:, heads]
        cuts = (crossing * c[None, :]).sum(axis=1)
    else:
        cuts = np.zeros(1 << k, dtype=np.int64)
    best = int(cuts.min())
    union = member[cuts == best].any(axis=0).astype(np.uint8)
    return best, union


# --------------------------------------------------------------------------
# Merged arc pairs and O4
# --------------------------------------------------------------------------

@dataclass
class PairGraph:
    n: int
    m: int
    s: int
    t: int
    row_ptr: np.ndarray   # int32[n+1]
    col: np.ndarray       # int32[A]
    twin: np.ndarray      # int32[A]
    cap: np.ndarray       # int32[A]  (current capacities, summed per direction)
    edge2arc: np.ndarray  # int32[m]  (-1 for self-loops)
    ecap: np.ndarray      # int32[m]  (current per-edge capacities)

    @property
    def A(self) -> int:
        return int(self.col.shape[0])

    @staticmethod
    def build(g, cap=None) -> "PairGraph":
        rp, col, _ = _csr(g)
        c = _cap_or(g, cap)
        L = lib()
        A = L.orc_pairs_count(g.n, col.shape[0], rp, col)
        if A < 0:
            raise MemoryError("oracle allocation failed")
        arp = np.zeros(g.n + 1, dtype=np.int32)
        acol = np.zeros(max(1, A), dtype=np.int32)
        atwin = np.zeros(max(1, A), dtype=np.int32)
        acap = np.zeros(max(1, A), dtype=np.int32)
        e2a = np.zeros(max(1, col.shape[0]), dtype=np.int32)
        rc = L.orc_pairs_build(g.n, col.shape[0], rp, col, c, arp, acol, atwin, acap, e2a)
        if rc == -2:
            raise OverflowError("summed pair capacity exceeds int32")
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        return PairGraph(g.n, col.shape[0], g.s, g.t, arp, acol[:A], atwin[:A], acap[:A],
                         e2a[: col.shape[0]], c.copy())

    def tails(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr))


def bfs_heights(pg: PairGraph, cf, e) -> np.ndarray:
    """Global-relabel heights of a residual state: 0 at t and at deficient
    vertices other than s, exact residual BFS distance to them elsewhere,
    |V| where no root is reachable (and always at s)."""
    h = np.zeros(pg.n, dtype=np.int32)
    lib().orc_paper_global_relabel(pg.n, pg.row_ptr, pg.col, pg.twin,
                                   np.ascontiguousarray(cf, dtype=np.int32),
                                   np.ascontiguousarray(e, dtype=np.int64), pg.s, pg.t, h)
    return h


def paper_value(e, s, t) -> int:
    e = np.ascontiguousarray(e, dtype=np.int64)
    return int(lib().orc_paper_value(e.shape[0], e, s, t))


class PaperSeq:
    """O4: the paper's static and dynamic push-relabel, sequential, on merged
    arc pairs.  State arrays are public so that tests can load a GPU state
    into them and replay one deterministic step."""

    def __init__(self, g, kernel_cycles: int | None = None, cap=None):
        self.pg = PairGraph.build(g, cap)
        self.kc = int(kernel_cycles) if kernel_cycles else max(1, int(round(g.m / g.n)))
        self.cf = np.zeros(self.pg.A, dtype=np.int32)
        self.e = np.zeros(self.pg.n, dtype=np.int64)
        self.h = np.zeros(self.pg.n, dtype=np.int32)
        self.stats = np.zeros(3, dtype=np.int64)

    # Alg. 1 lines 1-13
    def init(self):
        pg = self.pg
        lib().orc_paper_init(pg.n, pg.A, pg.row_ptr, pg.col, pg.twin, pg.cap, pg.s,
                             self.cf, self.e, self.h)

    def loop(self, max_iter: int = -1) -> bool:
        pg = self.pg
        rc = lib().orc_paper_loop(pg.n, pg.row_ptr, pg.col, pg.twin, self.cf, self.e, self.h,
                                  pg.s, pg.t, self.kc, int(max_iter), self.stats)
        return rc == 0

    def solve(self) -> int:
        self.init()
        if not self.loop():
            raise RuntimeError("unreachable: unbounded loop reported a limit")
        return self.value()

    # Alg. 5 + excess recomputation + source re-saturation (Alg. 4 lines 1-8)
    def apply_updates(self, ids, new_caps):
        pg = self.pg
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        new_caps = np.ascontiguousarray(new_caps, dtype=np.int32)
        if np.unique(ids).shape[0] != ids.shape[0]:
            raise ValueError("a batch is a set: edge ids must be distinct")
        lib().orc_paper_apply_updates(pg.n, pg.A, pg.row_ptr, pg.col, pg.twin, pg.cap,
                                      pg.edge2arc, pg.ecap, self.cf, self.e, pg.s, ids, new_caps,
                                      ids.shape[0])

    def update(self, ids, new_caps) -> int:
        self.apply_updates(ids, new_caps)
        if not self.loop():
            raise RuntimeError("unreachable: unbounded loop reported a limit")
        return self.value()

    def value(self) -> int:
        return paper_value(self.e, self.pg.s, self.pg.t)

    def source_side(self) -> np.ndarray:
        return (self.h >= self.pg.n).astype(np.uint8)


def validate(pg: PairGraph, cf, e, cap=None):
    """V.  Returns (code, value, side, pair_flow); code 0 means the state is a
    valid maximum preflow state whose completion is a valid flow of `value`
    certified by the cut `side`."""
    side = np.zeros(pg.n, dtype=np.uint8)
    val = C.c_int64(0)
    flow = np.zeros(max(1, pg.A), dtype=np.int64)
    capa = np.ascontiguousarray(pg.cap if cap is None else cap, dtype=np.int32)
    rc = lib().orc_validate(pg.n, pg.A, pg.row_ptr, pg.col, pg.twin, capa,
                            np.ascontiguousarray(cf, dtype=np.int32),
                            np.ascontiguousarray(e, dtype=np.int64), pg.s, pg.t, side,
                            C.byref(val), flow)
    return int(rc), int(val.value), side, flow[: pg.A]
