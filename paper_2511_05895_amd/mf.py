"""ctypes binding of libmf.so (include/mf.h): the same entry points, argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; there is no fallback path.  Importing this module raises when the
built library is missing."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_ESTATE, MF_ETIMEOUT = range(6)
MF_MODE_DATA, MF_MODE_TOPOLOGY = 0, 1
MF_FLAG_GAP = 1
_NAMES = {1: "MF_EINVAL", 2: "MF_ENOMEM", 3: "MF_EDEVICE", 4: "MF_ESTATE", 5: "MF_ETIMEOUT"}


class MfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class mf_csr_t(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p)]


class mf_opts_t(C.Structure):
    _fields_ = [("kernel_cycles", C.c_int32), ("mode", C.c_int32), ("grid_blocks", C.c_int32),
                ("device", C.c_int32), ("max_iterations", C.c_int64), ("time_budget_ms", C.c_int32),
                ("max_rounds", C.c_int32), ("relabel_budget", C.c_int32), ("rounds_per_level", C.c_int32),
                ("flags", C.c_int32), ("stall_rounds", C.c_int32), ("reserved", C.c_int32 * 2)]


class mf_stats_t(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "iterations", "global_relabels", "bfs_levels", "bfs_vertices", "bfs_arcs",
        "pr_vertex_cycles", "pr_arcs", "pushes", "relabels", "rie_arcs", "rie_saturations",
        "updates", "clamps", "source_pushes", "rounds", "loop_launches", "grid_blocks")] + [
        (name, C.c_double) for name in ("bfs_ms", "pr_ms", "rie_ms", "loop_kernel_ms", "call_ms")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MF_BATCH_MAX_CLASSES = 4


class mf_batch_opts_t(C.Structure):
    _fields_ = [("device", C.c_int32), ("time_budget_ms", C.c_int32), ("n_classes", C.c_int32),
                ("use_graph", C.c_int32), ("class_max_arcs", C.c_int64 * MF_BATCH_MAX_CLASSES),
                ("block", C.c_int32 * MF_BATCH_MAX_CLASSES),
                ("kernel_cycles", C.c_int32 * MF_BATCH_MAX_CLASSES), ("flags", C.c_int32),
                ("stall_rounds", C.c_int32), ("reserved", C.c_int32 * 2)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if hasattr(v, "__len__") else v
        return d


# Every symbol that include/mf.h declares, with its C signature.
_SIGS = {
    "mf_default_opts": (None, [C.POINTER(mf_opts_t)]),
    "mf_create": (C.c_int, [C.POINTER(mf_csr_t), C.c_void_p, C.c_int32, C.c_int32,
                            C.POINTER(mf_opts_t), C.POINTER(C.c_void_p)]),
    "mf_destroy": (None, [C.c_void_p]),
    "mf_last_error": (C.c_char_p, [C.c_void_p]),
    "mf_solve": (C.c_int, [C.c_void_p]),
    "mf_apply_updates": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "mf_apply_updates_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "mf_set_capacities": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "mf_resume": (C.c_int, [C.c_void_p]),
    "mf_flow_value": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "mf_min_cut": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "mf_set_max_iterations": (C.c_int, [C.c_void_p, C.c_int64]),
    "mf_get_stats": (C.c_int, [C.c_void_p, C.POINTER(mf_stats_t)]),
    "mf_num_arcs": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_cap_limit": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_export_graph": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mf_export_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "mf_get_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "mf_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_batch_default_opts": (None, [C.POINTER(mf_batch_opts_t)]),
    "mf_batch_create": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.POINTER(mf_batch_opts_t),
                                  C.POINTER(C.c_void_p)]),
    "mf_batch_destroy": (None, [C.c_void_p]),
    "mf_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "mf_batch_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_batch_get_opts": (C.c_int, [C.c_void_p, C.POINTER(mf_batch_opts_t)]),
    "mf_batch_set_opts": (C.c_int, [C.c_void_p, C.POINTER(mf_batch_opts_t)]),
    "mf_batch_solve": (C.c_int, [C.c_void_p]),
    "mf_batch_solve_class": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "mf_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(mf_batch_opts_t)]),
    "mf_batch_values": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_batch_num_arcs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_batch_last_ms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "mf_batch_min_cut": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]),
    "mf_batch_get_stats": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(mf_stats_t)]),
    "mf_batch_set_capacities": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2511_05895_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(rc, h=None):
    if rc != MF_OK:
        msg = lib().mf_last_error(h)
        raise MfError(rc, msg.decode() if msg else "")
    return rc


# ---------------- same names as the C-ABI ----------------

def mf_default_opts() -> mf_opts_t:
    o = mf_opts_t()
    lib().mf_default_opts(C.byref(o))
    return o


def mf_create(n, row_ptr, col, cap, s, t, opts: mf_opts_t | None = None):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    cap = np.ascontiguousarray(cap, dtype=np.int32)
    g = mf_csr_t(int(n), int(col.shape[0]), row_ptr.ctypes.data, col.ctypes.data)
    out = C.c_void_p()
    rc = lib().mf_create(C.byref(g), C.c_void_p(cap.ctypes.data), int(s), int(t),
                         C.byref(opts) if opts is not None else None, C.byref(out))
    _check(rc, None)
    return out


def mf_destroy(h):
    lib().mf_destroy(h)


def mf_last_error(h=None) -> str:
    msg = lib().mf_last_error(h)
    return msg.decode() if msg else ""


def mf_solve(h):
    return _check(lib().mf_solve(h), h)


def mf_apply_updates(h, edge_ids, new_caps):
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    caps = np.ascontiguousarray(new_caps, dtype=np.int32)
    if ids.shape != caps.shape:
        raise ValueError("edge_ids and new_caps differ in length")
    return _check(lib().mf_apply_updates(h, _ptr(ids), _ptr(caps), ids.shape[0]), h)


def mf_apply_updates_device(h, d_edge_ids_ptr: int, d_new_caps_ptr: int, k: int):
    return _check(lib().mf_apply_updates_device(h, C.c_void_p(d_edge_ids_ptr),
                                                C.c_void_p(d_new_caps_ptr), int(k)), h)


def mf_set_capacities(h, edge_ids, new_caps):
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    caps = np.ascontiguousarray(new_caps, dtype=np.int32)
    if ids.shape != caps.shape:
        raise ValueError("edge_ids and new_caps differ in length")
    return _check(lib().mf_set_capacities(h, _ptr(ids), _ptr(caps), ids.shape[0]), h)


def mf_resume(h):
    return _check(lib().mf_resume(h), h)


def mf_flow_value(h) -> int:
    v = C.c_int64()
    _check(lib().mf_flow_value(h, C.byref(v)), h)
    return int(v.value)


def mf_min_cut(h, n: int):
    side = np.zeros(n, dtype=np.uint8)
    cut = C.c_int64()
    _check(lib().mf_min_cut(h, _ptr(side), C.byref(cut)), h)
    return side, int(cut.value)


def mf_set_max_iterations(h, limit: int):
    return _check(lib().mf_set_max_iterations(h, int(limit)), h)


def mf_get_stats(h) -> dict:
    s = mf_stats_t()
    _check(lib().mf_get_stats(h, C.byref(s)), h)
    return s.as_dict()


def mf_num_arcs(h) -> int:
    a = C.c_int32()
    _check(lib().mf_num_arcs(h, C.byref(a)), h)
    return int(a.value)


def mf_cap_limit(h) -> int:
    a = C.c_int32()
    _check(lib().mf_cap_limit(h, C.byref(a)), h)
    return int(a.value)


def mf_export_graph(h, n: int, m: int):
    A = mf_num_arcs(h)
    rp = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(max(A, 1), dtype=np.int32)
    twin = np.zeros(max(A, 1), dtype=np.int32)
    e2a = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().mf_export_graph(h, _ptr(rp), _ptr(col), _ptr(twin), _ptr(e2a)), h)
    return rp, col[:A], twin[:A], e2a[:m]


def mf_export_state(h, n: int, m: int):
    A = mf_num_arcs(h)
    cap = np.zeros(max(A, 1), dtype=np.int32)
    cf = np.zeros(max(A, 1), dtype=np.int32)
    e = np.zeros(n, dtype=np.int64)
    hgt = np.zeros(n, dtype=np.int32)
    ecap = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().mf_export_state(h, _ptr(cap), _ptr(cf), _ptr(e), _ptr(hgt), _ptr(ecap)), h)
    return cap[:A], cf[:A], e, hgt, ecap[:m]


TRACE_FIELDS = ("levels", "active", "rounds", "reason", "relabels", "relabelled", "pushes", "last_delivery")


def mf_get_trace(h, max_phases: int = 256) -> np.ndarray:
    """int32[phases, 8] per-phase records of the last solving call."""
    out = np.zeros((max_phases, len(TRACE_FIELDS)), dtype=np.int32)
    n = C.c_int32()
    _check(lib().mf_get_trace(h, _ptr(out), max_phases, C.byref(n)), h)
    return out[: min(n.value, max_phases)]


def mf_set_stream(h, stream_ptr: int | None):
    return _check(lib().mf_set_stream(h, C.c_void_p(stream_ptr) if stream_ptr else None), h)


# ---------------- convenience wrapper ----------------

class MaxFlow:
    """Owns one handle.  g: object with n, row_ptr, col, cap, s, t."""

    def __init__(self, g, kernel_cycles=0, mode=MF_MODE_DATA, grid_blocks=0, max_iterations=-1,
                 device=0, cap=None, time_budget_ms=0, max_rounds=0, relabel_budget=0,
                 rounds_per_level=0, flags=0, stall_rounds=0):
        o = mf_default_opts()
        o.time_budget_ms = time_budget_ms
        o.max_rounds = max_rounds
        o.relabel_budget = relabel_budget
        o.rounds_per_level = rounds_per_level
        o.flags = flags
        o.stall_rounds = stall_rounds
        o.kernel_cycles = kernel_cycles
        o.mode = mode
        o.grid_blocks = grid_blocks
        o.max_iterations = max_iterations
        o.device = device
        self.n, self.m = int(g.n), int(g.col.shape[0])
        self.h = mf_create(g.n, g.row_ptr, g.col, g.cap if cap is None else cap, g.s, g.t, o)

    def close(self):
        if self.h:
            mf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self) -> int:
        mf_solve(self.h)
        return mf_flow_value(self.h)

    def update(self, edge_ids, new_caps) -> int:
        mf_apply_updates(self.h, edge_ids, new_caps)
        return mf_flow_value(self.h)

    def update_device(self, ids_tensor, caps_tensor) -> int:
        k = int(ids_tensor.numel())
        mf_apply_updates_device(self.h, ids_tensor.data_ptr(), caps_tensor.data_ptr(), k)
        return mf_flow_value(self.h)

    def set_capacities(self, edge_ids, new_caps):
        mf_set_capacities(self.h, edge_ids, new_caps)

    def resume(self) -> int:
        mf_resume(self.h)
        return mf_flow_value(self.h)

    def value(self) -> int:
        return mf_flow_value(self.h)

    def min_cut(self):
        return mf_min_cut(self.h, self.n)

    def stats(self) -> dict:
        return mf_get_stats(self.h)

    def trace(self) -> np.ndarray:
        return mf_get_trace(self.h)

    def set_max_iterations(self, limit: int):
        mf_set_max_iterations(self.h, limit)

    def export_graph(self):
        return mf_export_graph(self.h, self.n, self.m)

    def export_state(self):
        return mf_export_state(self.h, self.n, self.m)

    @property
    def num_arcs(self) -> int:
        return mf_num_arcs(self.h)

    @property
    def cap_limit(self) -> int:
        return mf_cap_limit(self.h)


# ---------------- batched solve (mf_batch_*) ----------------

def _bcheck(rc, b=None):
    if rc != MF_OK:
        msg = lib().mf_batch_last_error(b)
        raise MfError(rc, msg.decode() if msg else "")
    return rc


def mf_batch_default_opts() -> mf_batch_opts_t:
    o = mf_batch_opts_t()
    lib().mf_batch_default_opts(C.byref(o))
    return o


def mf_batch_create(graphs, caps=None, opts: mf_batch_opts_t | None = None):
    """graphs: objects with n, row_ptr, col, cap, s, t; caps: optional list of
    per-instance capacity arrays.  Packs them block-diagonally."""
    cnt = len(graphs)
    n = np.array([g.n for g in graphs], dtype=np.int32)
    m = np.array([g.col.shape[0] for g in graphs], dtype=np.int64)
    rp = np.concatenate([np.asarray(g.row_ptr, dtype=np.int64) for g in graphs]) if cnt else np.zeros(0, np.int64)
    col = np.concatenate([np.asarray(g.col, dtype=np.int32) for g in graphs] + [np.zeros(0, np.int32)])
    cp = np.concatenate([np.asarray(g.cap if caps is None else caps[i], dtype=np.int32)
                         for i, g in enumerate(graphs)] + [np.zeros(0, np.int32)])
    s = np.array([g.s for g in graphs], dtype=np.int32)
    t = np.array([g.t for g in graphs], dtype=np.int32)
    out = C.c_void_p()
    rc = lib().mf_batch_create(cnt, _ptr(n), _ptr(m), _ptr(rp), _ptr(col), _ptr(cp), _ptr(s), _ptr(t),
                               C.byref(opts) if opts is not None else None, C.byref(out))
    _bcheck(rc, None)
    return out


def mf_batch_destroy(b):
    lib().mf_batch_destroy(b)


def mf_batch_solve(b):
    return _bcheck(lib().mf_batch_solve(b), b)


def mf_batch_solve_class(b, cls: int) -> float:
    ms = C.c_double()
    _bcheck(lib().mf_batch_solve_class(b, int(cls), C.byref(ms)), b)
    return float(ms.value)


def mf_batch_autotune(b, repeats: int = 3) -> mf_batch_opts_t:
    o = mf_batch_opts_t()
    _bcheck(lib().mf_batch_autotune(b, int(repeats), C.byref(o)), b)
    return o


def mf_batch_get_opts(b) -> mf_batch_opts_t:
    o = mf_batch_opts_t()
    _bcheck(lib().mf_batch_get_opts(b, C.byref(o)), b)
    return o


def mf_batch_set_opts(b, o: mf_batch_opts_t):
    return _bcheck(lib().mf_batch_set_opts(b, C.byref(o)), b)


def mf_batch_count(b) -> int:
    c = C.c_int32()
    _bcheck(lib().mf_batch_count(b, C.byref(c)), b)
    return int(c.value)


def mf_batch_values(b) -> np.ndarray:
    out = np.zeros(mf_batch_count(b), dtype=np.int64)
    _bcheck(lib().mf_batch_values(b, _ptr(out)), b)
    return out


def mf_batch_num_arcs(b) -> np.ndarray:
    out = np.zeros(mf_batch_count(b), dtype=np.int64)
    _bcheck(lib().mf_batch_num_arcs(b, _ptr(out)), b)
    return out


def mf_batch_last_ms(b) -> float:
    ms = C.c_double()
    _bcheck(lib().mf_batch_last_ms(b, C.byref(ms)), b)
    return float(ms.value)


def mf_batch_min_cut(b, i: int, n: int):
    side = np.zeros(n, dtype=np.uint8)
    cut = C.c_int64()
    _bcheck(lib().mf_batch_min_cut(b, int(i), _ptr(side), C.byref(cut)), b)
    return side, int(cut.value)


def mf_batch_get_stats(b, i: int) -> dict:
    s = mf_stats_t()
    _bcheck(lib().mf_batch_get_stats(b, int(i), C.byref(s)), b)
    return s.as_dict()


def mf_batch_set_capacities(b, i: int, edge_ids, new_caps):
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    caps = np.ascontiguousarray(new_caps, dtype=np.int32)
    if ids.shape != caps.shape:
        raise ValueError("edge_ids and new_caps differ in length")
    return _bcheck(lib().mf_batch_set_capacities(b, int(i), _ptr(ids), _ptr(caps), ids.shape[0]), b)


class Batch:
    """Owns one batch of independent instances solved together."""

    def __init__(self, graphs, caps=None, n_classes=None, class_max_arcs=None, block=None,
                 kernel_cycles=None, use_graph=True, time_budget_ms=0, flags=0, stall_rounds=0, device=0):
        o = mf_batch_default_opts()
        o.device = device
        o.time_budget_ms = time_budget_ms
        o.use_graph = 1 if use_graph else 0
        o.flags = flags
        o.stall_rounds = stall_rounds
        if n_classes is not None:
            o.n_classes = n_classes
        for name, val in (("class_max_arcs", class_max_arcs), ("block", block), ("kernel_cycles", kernel_cycles)):
            if val is not None:
                arr = getattr(o, name)
                for i, x in enumerate(val):
                    arr[i] = x
        self.ns = [int(g.n) for g in graphs]
        self.b = mf_batch_create(graphs, caps, o)

    def close(self):
        if self.b:
            mf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self) -> np.ndarray:
        mf_batch_solve(self.b)
        return mf_batch_values(self.b)

    def values(self) -> np.ndarray:
        return mf_batch_values(self.b)

    def solve_class(self, cls: int) -> float:
        return mf_batch_solve_class(self.b, cls)

    def autotune(self, repeats: int = 3) -> dict:
        return mf_batch_autotune(self.b, repeats).as_dict()

    def opts(self) -> dict:
        return mf_batch_get_opts(self.b).as_dict()

    def set_opts(self, **kw):
        o = mf_batch_get_opts(self.b)
        for k, v in kw.items():
            if hasattr(v, "__len__"):
                arr = getattr(o, k)
                for i, x in enumerate(v):
                    arr[i] = x
            else:
                setattr(o, k, v)
        mf_batch_set_opts(self.b, o)

    def last_ms(self) -> float:
        return mf_batch_last_ms(self.b)

    def num_arcs(self) -> np.ndarray:
        return mf_batch_num_arcs(self.b)

    def min_cut(self, i: int):
        # an out-of-range index is rejected by the library (MF_EINVAL)
        return mf_batch_min_cut(self.b, i, self.ns[i] if 0 <= i < len(self.ns) else 0)

    def stats(self, i: int) -> dict:
        return mf_batch_get_stats(self.b, i)

    def set_capacities(self, i: int, edge_ids, new_caps):
        mf_batch_set_capacities(self.b, i, edge_ids, new_caps)


# Load at import: a missing or broken library is an ImportError, never a fallback.
lib()
