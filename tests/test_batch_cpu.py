"""Batched-solve entry points without a GPU: options and every instance are
checked on the host before any device work, and errors name the instance."""
import ctypes as C

import numpy as np
import pytest

from tests.graphs import from_edges


@pytest.fixture(scope="module")
def mf():
    from paper_2511_05895_amd import mf as m
    return m


def _two_instances():
    a = from_edges(3, [(0, 1, 4), (1, 2, 3)], 0, 2)
    b = from_edges(4, [(0, 1, 2), (1, 3, 2), (0, 2, 1), (2, 3, 5)], 0, 3)
    return [a, b]


def test_default_opts(mf):
    o = mf.mf_batch_default_opts()
    assert o.n_classes == 3 and o.use_graph == 1
    assert list(o.class_max_arcs)[:2] == [32768, 262144]
    assert list(o.block)[:3] == [256, 1024, 1024]
    assert list(o.kernel_cycles) == [0] * mf.MF_BATCH_MAX_CLASSES


@pytest.mark.parametrize("field,value,expect", [
    ("block", [300, 1024, 1024, 1024], "block must be"),
    ("n_classes", 0, "n_classes"),
    ("n_classes", 5, "n_classes"),
    ("class_max_arcs", [100, 50, 0, 0], "ascending"),
    ("kernel_cycles", [-1, 0, 0, 0], "kernel_cycles"),
    ("flags", 8, "unknown flags"),
    ("use_graph", 2, "use_graph"),
    ("reserved", [0, 3], "reserved"),
    ("time_budget_ms", -5, "time_budget_ms"),
])
def test_create_rejects_bad_options(mf, field, value, expect):
    o = mf.mf_batch_default_opts()
    if isinstance(value, list):
        arr = getattr(o, field)
        for i, x in enumerate(value):
            arr[i] = x
    else:
        setattr(o, field, value)
    with pytest.raises(mf.MfError) as ei:
        mf.mf_batch_create(_two_instances(), None, o)
    assert ei.value.code == mf.MF_EINVAL
    assert expect in str(ei.value)


@pytest.mark.parametrize("case,expect", [
    ("s==t", "instance 1: s == t"),
    ("col", "instance 1: col out of range"),
    ("neg", "instance 0: negative capacity"),
    ("n<2", "instance 0: n must be"),
])
def test_create_rejects_bad_instances(mf, case, expect):
    gs = _two_instances()
    caps = [g.cap.copy() for g in gs]
    if case == "s==t":
        gs[1].t = gs[1].s
    elif case == "col":
        gs[1].col = gs[1].col.copy()
        gs[1].col[0] = 9
    elif case == "neg":
        caps[0][1] = -1
    elif case == "n<2":
        g = from_edges(2, [], 0, 1)
        g.n = 1
        g.row_ptr = np.zeros(2, np.int64)
        g.t = 0
        gs[0] = g
        caps[0] = g.cap
    with pytest.raises(mf.MfError) as ei:
        mf.mf_batch_create(gs, caps)
    assert ei.value.code == mf.MF_EINVAL
    assert expect in str(ei.value)


def test_create_rejects_empty_batch(mf):
    out = C.c_void_p()
    rc = mf.lib().mf_batch_create(0, None, None, None, None, None, None, None, None, C.byref(out))
    assert rc == mf.MF_EINVAL
    assert "count" in mf.lib().mf_batch_last_error(None).decode()
