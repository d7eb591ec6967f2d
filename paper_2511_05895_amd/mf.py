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

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_ESTATE, MF_ETIMEOUT, MF_EPENDING, MF_EBUSY = range(8)
MF_MODE_DATA, MF_MODE_TOPOLOGY = 0, 1
MF_FLAG_GAP = 1
MF_FLAG_PUSH_PULL = 2
MF_FLAG_DEBUG_CHECKS = 4
MF_FLAG_SCAN_FIRST = 8
MF_FLAG_GLOBAL_ONLY = 16
MF_ORDER_AUTO, MF_ORDER_INPUT, MF_ORDER_DEGREE = 0, 1, 2
MF_NOALLOC_MAX_UPDATES = 1 << 20  # batch limit of mf_apply_updates_noalloc
_NAMES = {1: "MF_EINVAL", 2: "MF_ENOMEM", 3: "MF_EDEVICE", 4: "MF_ESTATE", 5: "MF_ETIMEOUT",
          6: "MF_EPENDING", 7: "MF_EBUSY"}


class MfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class mf_csr_t(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mf_opts_t(C.Structure):
    _fields_ = [("kernel_cycles", C.c_int32), ("mode", C.c_int32), ("grid_blocks", C.c_int32),
                ("device", C.c_int32), ("max_iterations", C.c_int64), ("time_budget_ms", C.c_int32),
                ("max_rounds", C.c_int32), ("relabel_budget", C.c_int32), ("rounds_per_level", C.c_int32),
                ("flags", C.c_int32), ("stall_rounds", C.c_int32), ("solo_items", C.c_int32),
                ("lazy_items", C.c_int32),
                ("bottom_up", C.c_int32), ("vertex_order", C.c_int32), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", C.c_void_p)]


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


class mf_server_opts_t(C.Structure):
    _fields_ = [("device", C.c_int32), ("workers", C.c_int32), ("memory_budget", C.c_int64),
                ("max_group_edges", C.c_int64), ("max_group_requests", C.c_int32),
                ("reserved0", C.c_int32), ("max_pending_bytes", C.c_int64), ("reserved", C.c_int32 * 2)]


class mf_result_t(C.Structure):
    _fields_ = [("status", C.c_int32), ("graph", C.c_int32), ("request", C.c_int64), ("value", C.c_int64),
                ("version", C.c_int64), ("seq", C.c_int64), ("group_size", C.c_int64),
                ("submit_ms", C.c_double), ("start_ms", C.c_double), ("done_ms", C.c_double)]

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
    "mf_apply_updates_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "mf_set_capacities": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "mf_resume": (C.c_int, [C.c_void_p]),
    "mf_flow_value": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "mf_edge_flow": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_min_cut": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "mf_set_max_iterations": (C.c_int, [C.c_void_p, C.c_int64]),
    "mf_get_stats": (C.c_int, [C.c_void_p, C.POINTER(mf_stats_t)]),
    "mf_num_arcs": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_cap_limit": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_export_graph": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mf_export_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "mf_get_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "mf_import_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
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
    "mf_estimate_device_bytes": (C.c_int64, [C.c_int32, C.c_int64]),
    "mf_policy_last_error": (C.c_char_p, []),
    "mf_policy_num_params": (C.c_int32, []),
    "mf_policy_create": (C.c_int, [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]),
    "mf_policy_destroy": (None, [C.c_void_p]),
    "mf_policy_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_policy_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mf_policy_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "mf_policy_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_float)]),
    "mf_policy_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                  C.c_float, C.POINTER(C.c_float)]),
    "mf_set_policy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float, C.c_uint64,
                                C.c_int32]),
    "mf_get_policy_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "mf_server_default_opts": (None, [C.POINTER(mf_server_opts_t)]),
    "mf_server_last_error": (C.c_char_p, []),
    "mf_server_create": (C.c_int, [C.POINTER(mf_server_opts_t), C.POINTER(C.c_void_p)]),
    "mf_server_destroy": (None, [C.c_void_p]),
    "mf_server_add_graph": (C.c_int, [C.c_void_p, C.POINTER(mf_csr_t), C.c_void_p, C.c_int32, C.c_int32,
                                      C.POINTER(mf_opts_t), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "mf_server_remove_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "mf_server_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "mf_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(mf_result_t)]),
    "mf_server_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "mf_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(mf_result_t)]),
    "mf_server_drain": (C.c_int, [C.c_void_p]),
    "mf_server_graph_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mf_server_memory": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]),
    "mf_server_load": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int64)]),
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


def mf_apply_updates_noalloc(h, edge_ids, new_caps):
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    caps = np.ascontiguousarray(new_caps, dtype=np.int32)
    if ids.shape != caps.shape:
        raise ValueError("edge_ids and new_caps differ in length")
    return _check(lib().mf_apply_updates_noalloc(h, _ptr(ids), _ptr(caps), ids.shape[0]), h)


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


def mf_edge_flow(h, m: int) -> np.ndarray:
    flow = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().mf_edge_flow(h, _ptr(flow)), h)
    return flow[:m]


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


def mf_import_state(h, cap, cf, e, ecap):
    cap = np.ascontiguousarray(cap, dtype=np.int32)
    cf = np.ascontiguousarray(cf, dtype=np.int32)
    e = np.ascontiguousarray(e, dtype=np.int64)
    ecap = np.ascontiguousarray(ecap, dtype=np.int32)
    return _check(lib().mf_import_state(h, _ptr(cap), _ptr(cf), _ptr(e), _ptr(ecap)), h)


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

class TorchAllocator:
    """Device memory for a handle from torch's caching allocator: each block
    is a uint8 tensor kept alive until the library frees it."""

    def __init__(self, device=0, fail_after=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        self.live = {}
        self.fail_after = fail_after  # refuse allocations after this many (tests)
        self.calls = 0

    def alloc(self, nbytes: int) -> int:
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return 0
        t = self._torch.empty(max(nbytes, 1), dtype=self._torch.uint8, device=self.device)
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def free(self, ptr: int):
        self.live.pop(ptr, None)


class MaxFlow:
    """Owns one handle.  g: object with n, row_ptr, col, cap, s, t."""

    def __init__(self, g, kernel_cycles=0, mode=MF_MODE_DATA, grid_blocks=0, max_iterations=-1,
                 device=0, cap=None, time_budget_ms=0, max_rounds=0, relabel_budget=0,
                 rounds_per_level=0, flags=0, stall_rounds=0, solo_items=0, lazy_items=0, bottom_up=0,
                 vertex_order=0,
                 allocator=None):
        """allocator: optional object with alloc(nbytes) -> device address (0
        on failure) and free(address); the handle's device memory then comes
        from it (e.g. TorchAllocator)."""
        o = mf_default_opts()
        self._alloc_cbs = None
        if allocator is not None:
            # the callbacks must outlive the handle: kept on the object
            self._alloc_cbs = (ALLOC_FN(lambda nbytes, ctx: allocator.alloc(int(nbytes)) or None),
                               FREE_FN(lambda ptr, ctx: allocator.free(int(ptr))))
            o.dev_alloc, o.dev_free = self._alloc_cbs
        o.solo_items = solo_items
        o.lazy_items = lazy_items
        o.bottom_up = bottom_up
        o.vertex_order = vertex_order
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

    def update_noalloc(self, edge_ids, new_caps) -> int:
        mf_apply_updates_noalloc(self.h, edge_ids, new_caps)
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

    def edge_flow(self) -> np.ndarray:
        return mf_edge_flow(self.h, self.m)

    def stats(self) -> dict:
        return mf_get_stats(self.h)

    def trace(self) -> np.ndarray:
        return mf_get_trace(self.h)

    def set_policy(self, policy=None, mode=0, margin=0.0, explore=0.0, seed=0,
                   action=0):
        mf_set_policy(self.h, policy, mode, margin, explore, seed, action)

    def policy_trace(self) -> np.ndarray:
        return mf_get_policy_trace(self.h)

    def set_max_iterations(self, limit: int):
        mf_set_max_iterations(self.h, limit)

    def export_graph(self):
        return mf_export_graph(self.h, self.n, self.m)

    def export_state(self):
        return mf_export_state(self.h, self.n, self.m)

    def import_state(self, cap, cf, e, ecap):
        mf_import_state(self.h, cap, cf, e, ecap)

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


# ---------------- learned phase schedule (mf_policy_*, mf_set_policy) ----------------

POLICY_FEATURES, POLICY_HIDDEN, POLICY_ACTIONS = 16, 32, 8
MF_POLICY_FIXED, MF_POLICY_LEARNED, MF_POLICY_EXPLORE, MF_POLICY_FORCED = range(4)
MF_POLICY_PER_CALL = 16


def _pcheck(rc):
    if rc != MF_OK:
        msg = lib().mf_policy_last_error()
        raise MfError(rc, msg.decode() if msg else "")
    return rc


class Policy:
    """The value network of the learned phase schedule (device parameters)."""

    def __init__(self, seed: int = 0, device: int = 0):
        out = C.c_void_p()
        _pcheck(lib().mf_policy_create(int(device), int(seed) & (2**64 - 1), C.byref(out)))
        self.p = out
        self.n_params = int(lib().mf_policy_num_params())

    def close(self):
        if self.p:
            lib().mf_policy_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _pcheck(lib().mf_policy_get_params(self.p, _ptr(out)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.shape != (self.n_params,):
            raise ValueError("wrong parameter count")
        _pcheck(lib().mf_policy_set_params(self.p, _ptr(theta)))

    def forward(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, POLICY_FEATURES)
        Q = np.zeros((X.shape[0], POLICY_ACTIONS), dtype=np.float32)
        _pcheck(lib().mf_policy_forward(self.p, _ptr(X), X.shape[0], _ptr(Q)))
        return Q

    def gradient(self, X, actions, targets):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, POLICY_FEATURES)
        a = np.ascontiguousarray(actions, dtype=np.int32)
        y = np.ascontiguousarray(targets, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        _pcheck(lib().mf_policy_gradient(self.p, _ptr(X), _ptr(a), _ptr(y), X.shape[0], _ptr(g), C.byref(loss)))
        return float(loss.value), g

    def train(self, X, actions, targets, steps: int = 500, lr: float = 3e-3) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, POLICY_FEATURES)
        a = np.ascontiguousarray(actions, dtype=np.int32)
        y = np.ascontiguousarray(targets, dtype=np.float32)
        loss = C.c_float()
        _pcheck(lib().mf_policy_train(self.p, _ptr(X), _ptr(a), _ptr(y), X.shape[0], int(steps), float(lr),
                                      C.byref(loss)))
        return float(loss.value)


def mf_set_policy(h, policy: "Policy | None", mode: int, margin: float = 0.0, explore: float = 0.0,
                  seed: int = 0, action: int = 0):
    return _check(lib().mf_set_policy(h, policy.p if policy is not None else None, int(mode), float(margin),
                                      float(explore), int(seed) & (2**64 - 1), int(action)), h)


def mf_get_policy_trace(h, max_phases: int = 256) -> np.ndarray:
    """float32[phases, 18]: features, action taken, phase duration (ms)."""
    out = np.zeros((max_phases, POLICY_FEATURES + 2), dtype=np.float32)
    n = C.c_int32()
    _check(lib().mf_get_policy_trace(h, _ptr(out), max_phases, C.byref(n)), h)
    return out[: min(n.value, max_phases)]


# ---------------- serving runtime (mf_server_*) ----------------

def _scheck(rc):
    if rc not in (MF_OK, MF_EPENDING):
        msg = lib().mf_server_last_error()
        raise MfError(rc, msg.decode() if msg else "")
    return rc


def mf_estimate_device_bytes(n: int, m: int) -> int:
    return int(lib().mf_estimate_device_bytes(int(n), int(m)))


def mf_server_default_opts() -> mf_server_opts_t:
    o = mf_server_opts_t()
    lib().mf_server_default_opts(C.byref(o))
    return o


def mf_server_create(opts: mf_server_opts_t | None = None):
    out = C.c_void_p()
    _scheck(lib().mf_server_create(C.byref(opts) if opts is not None else None, C.byref(out)))
    return out


def mf_server_destroy(s):
    lib().mf_server_destroy(s)


def mf_server_add_graph(s, g, cap=None, opts: mf_opts_t | None = None):
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    cp = np.ascontiguousarray(g.cap if cap is None else cap, dtype=np.int32)
    csr = mf_csr_t(int(g.n), int(col.shape[0]), row_ptr.ctypes.data, col.ctypes.data)
    gid = C.c_int32()
    val = C.c_int64()
    _scheck(lib().mf_server_add_graph(s, C.byref(csr), _ptr(cp), int(g.s), int(g.t),
                                      C.byref(opts) if opts is not None else None, C.byref(gid), C.byref(val)))
    return int(gid.value), int(val.value)


def mf_server_remove_graph(s, graph_id: int):
    return _scheck(lib().mf_server_remove_graph(s, int(graph_id)))


def mf_server_submit(s, graph_id: int, edge_ids, new_caps) -> int:
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    caps = np.ascontiguousarray(new_caps, dtype=np.int32)
    if ids.shape != caps.shape:
        raise ValueError("edge_ids and new_caps differ in length")
    rid = C.c_int64()
    _scheck(lib().mf_server_submit(s, int(graph_id), _ptr(ids), _ptr(caps), ids.shape[0], C.byref(rid)))
    return int(rid.value)


def mf_server_poll(s, request_id: int):
    r = mf_result_t()
    rc = _scheck(lib().mf_server_poll(s, int(request_id), C.byref(r)))
    return None if rc == MF_EPENDING else r.as_dict()


def mf_server_release(s, request_id: int) -> bool:
    """True when released, False while the request is still pending."""
    rc = _scheck(lib().mf_server_release(s, int(request_id)))
    return rc == MF_OK


def mf_server_wait(s, request_id: int) -> dict:
    r = mf_result_t()
    _scheck(lib().mf_server_wait(s, int(request_id), C.byref(r)))
    return r.as_dict()


def mf_server_drain(s):
    return _scheck(lib().mf_server_drain(s))


def mf_server_graph_info(s, graph_id: int):
    v = C.c_int64()
    val = C.c_int64()
    _scheck(lib().mf_server_graph_info(s, int(graph_id), C.byref(v), C.byref(val)))
    return int(v.value), int(val.value)


def mf_server_memory(s):
    r, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _scheck(lib().mf_server_memory(s, C.byref(r), C.byref(b), C.byref(c)))
    return {"reserved": int(r.value), "budget": int(b.value), "commits": int(c.value)}


def mf_server_load(s):
    pb, su, sl, rs = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
    _scheck(lib().mf_server_load(s, C.byref(pb), C.byref(su), C.byref(sl), C.byref(rs)))
    return {"pending_bytes": int(pb.value), "slots_used": int(su.value), "slots": int(sl.value),
            "resumed": int(rs.value)}


class Server:
    """Owns one serving runtime."""

    def __init__(self, workers=4, memory_budget=0, max_group_edges=1 << 20, max_group_requests=64, device=0,
                 max_pending_bytes=0):
        o = mf_server_default_opts()
        o.device = device
        o.workers = workers
        o.memory_budget = memory_budget
        o.max_group_edges = max_group_edges
        o.max_group_requests = max_group_requests
        o.max_pending_bytes = max_pending_bytes
        self.s = mf_server_create(o)

    def close(self):
        if self.s:
            mf_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_graph(self, g, cap=None, **opts):
        o = None
        if opts:
            o = mf_default_opts()
            for k, v in opts.items():
                setattr(o, k, v)
        return mf_server_add_graph(self.s, g, cap, o)

    def remove_graph(self, graph_id: int):
        mf_server_remove_graph(self.s, graph_id)

    def submit(self, graph_id: int, edge_ids, new_caps) -> int:
        return mf_server_submit(self.s, graph_id, edge_ids, new_caps)

    def poll(self, request_id: int):
        return mf_server_poll(self.s, request_id)

    def wait(self, request_id: int) -> dict:
        return mf_server_wait(self.s, request_id)

    def release(self, request_id: int) -> bool:
        return mf_server_release(self.s, request_id)

    def drain(self):
        mf_server_drain(self.s)

    def graph_info(self, graph_id: int):
        return mf_server_graph_info(self.s, graph_id)

    def memory(self) -> dict:
        return mf_server_memory(self.s)

    def load(self) -> dict:
        return mf_server_load(self.s)


# Load at import: a missing or broken library is an ImportError, never a fallback.
lib()
