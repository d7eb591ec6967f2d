"""The C-ABI library without a GPU: it loads, exports every symbol that
include/mf.h declares, and rejects bad arguments on the host before any
device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mf.h")).read()
    return re.findall(r"MF_API\s+[\w\s\*]+?\b(mf_\w+)\s*\(", text)


def test_header_declares_the_core_calls():
    names = set(_declared_symbols())
    for core in ("mf_create", "mf_solve", "mf_apply_updates", "mf_flow_value", "mf_min_cut"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2511_05895_amd import mf
    lib = C.CDLL(mf.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
        assert name in mf._SIGS, f"binding lacks {name}"


def _create(n, rp, col, cap, s, t, opts=None):
    from paper_2511_05895_amd import mf
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    cap = np.ascontiguousarray(cap, dtype=np.int32)
    g = mf.mf_csr_t(n, col.shape[0], rp.ctypes.data, col.ctypes.data)
    out = C.c_void_p()
    rc = mf.lib().mf_create(C.byref(g), C.c_void_p(cap.ctypes.data), s, t,
                            C.byref(opts) if opts is not None else None, C.byref(out))
    return rc, out, mf.mf_last_error(None)


@pytest.mark.parametrize("case,expect", [
    ("n<2", "n must be"),
    ("s==t", "s == t"),
    ("s range", "out of range"),
    ("col range", "col out of range"),
    ("neg cap", "negative capacity"),
    ("row_ptr", "row_ptr"),
    ("mode", "unknown mode"),
    ("vertex order", "unknown vertex_order"),
    ("cap limit", "per-edge limit"),
    ("flags", "unknown flags"),
    ("alloc pair", "go together"),
])
def test_create_rejects_bad_arguments(case, expect):
    from paper_2511_05895_amd import mf
    n, rp, col, cap, s, t = 3, [0, 1, 2, 2], [1, 2], [5, 5], 0, 2
    opts = None
    if case == "n<2":
        n, rp = 1, [0, 2]
    elif case == "s==t":
        t = 0
    elif case == "s range":
        s = 7
    elif case == "col range":
        col = [1, 9]
    elif case == "neg cap":
        cap = [5, -1]
    elif case == "row_ptr":
        rp = [0, 2, 1, 2]
    elif case == "mode":
        opts = mf.mf_default_opts()
        opts.mode = 7
    elif case == "vertex order":
        opts = mf.mf_default_opts()
        opts.vertex_order = 3
    elif case == "cap limit":
        cap = [5, 1 << 30]
    elif case == "flags":
        opts = mf.mf_default_opts()
        opts.flags = 64
    elif case == "alloc pair":
        opts = mf.mf_default_opts()
        opts.dev_alloc = mf.ALLOC_FN(lambda nbytes, ctx: None)
    rc, h, msg = _create(n, rp, col, cap, s, t, opts)
    assert rc == mf.MF_EINVAL and not h.value
    assert expect in msg


def test_default_opts():
    from paper_2511_05895_amd import mf
    o = mf.mf_default_opts()
    assert (o.kernel_cycles, o.mode, o.grid_blocks, o.device, o.max_iterations) == (0, 0, 0, 0, -1)
