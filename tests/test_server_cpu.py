"""Serving runtime without a GPU: option checks happen before any device
call, and the admission estimate is plain host arithmetic."""
import ctypes as C

import pytest


@pytest.fixture(scope="module")
def mf():
    from paper_2511_05895_amd import mf as m
    return m


def test_default_opts(mf):
    o = mf.mf_server_default_opts()
    assert o.workers == 4 and o.max_group_edges == 1 << 20 and o.max_group_requests == 64
    assert o.memory_budget == 0 and o.max_pending_bytes == 1 << 30


@pytest.mark.parametrize("field,value,expect", [
    ("workers", 0, "workers"),
    ("workers", 65, "workers"),
    ("memory_budget", -1, "memory_budget"),
    ("max_group_edges", 0, "max_group_edges"),
    ("max_group_requests", 0, "max_group_requests"),
    ("max_pending_bytes", -1, "max_pending_bytes"),
    ("device", -1, "device"),
])
def test_create_rejects_bad_options(mf, field, value, expect):
    o = mf.mf_server_default_opts()
    setattr(o, field, value)
    with pytest.raises(mf.MfError) as ei:
        mf.mf_server_create(o)
    assert ei.value.code == mf.MF_EINVAL and expect in str(ei.value)


@pytest.mark.parametrize("which", ["reserved0", "reserved"])
def test_create_rejects_reserved(mf, which):
    o = mf.mf_server_default_opts()
    if which == "reserved0":
        o.reserved0 = 1
    else:
        o.reserved[1] = 1
    with pytest.raises(mf.MfError) as ei:
        mf.mf_server_create(o)
    assert ei.value.code == mf.MF_EINVAL


def test_estimate_device_bytes(mf):
    assert mf.mf_estimate_device_bytes(-1, 5) == -1
    small = mf.mf_estimate_device_bytes(1000, 8000)
    # every per-arc and per-vertex array is counted: at least 16 B per merged arc
    # (bounded by 2m), 12 B per edge and 44 B per vertex
    assert small >= 16 * 16000 + 12 * 8000 + 44 * 1000
    assert mf.mf_estimate_device_bytes(2000, 8000) > small
    assert mf.mf_estimate_device_bytes(1000, 16000) > small
    # C5 scale: 4M vertices, 64M edges -> a few GB, far below one GPU's memory
    c5 = mf.mf_estimate_device_bytes(1 << 22, 1 << 26)
    assert 2 << 30 < c5 < 6 << 30


def test_calls_reject_null_server(mf):
    r = mf.mf_result_t()
    assert mf.lib().mf_server_poll(None, 1, C.byref(r)) == mf.MF_EINVAL
    assert mf.lib().mf_server_drain(None) == mf.MF_EINVAL
    assert mf.lib().mf_server_release(None, 1) == mf.MF_EINVAL
    rid = C.c_int64()
    assert mf.lib().mf_server_submit(None, 0, None, None, 0, C.byref(rid)) == mf.MF_EINVAL
