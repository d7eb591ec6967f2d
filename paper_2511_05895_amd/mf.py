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


# Load at import: a missing or broken library is an ImportError, never a fallback.
lib()
