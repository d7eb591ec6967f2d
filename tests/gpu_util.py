"""Shared checks for the GPU parity tests: every result of the HIP path is
compared with the CPU oracle on the same seeded input."""
from __future__ import annotations

import time

import numpy as np

import oracle as O


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def check_layout(F, g, cap_now):
    """The device arc-pair layout equals the oracle's merged layout bit for bit."""
    pg = O.PairGraph.build(g, cap_now)
    rp, col, twin, e2a = F.export_graph()
    assert np.array_equal(rp, pg.row_ptr)
    assert np.array_equal(col, pg.col)
    assert np.array_equal(twin, pg.twin)
    assert np.array_equal(e2a, pg.edge2arc)
    return pg


def check_solved(F, g, cap_now, value=None, full=True, oracle="dinic", exact_heights=True):
    """Value and canonical cut equal the oracle's; the exported residual state
    passes the validator (and its completion is a valid flow of that value);
    the final heights are the exact global-relabel heights of that state
    (exact_heights; otherwise only their cut, h >= n, is compared)."""
    v = F.value()
    t0 = time.time()
    big = g.n > 100000
    if big:
        log(f"checking n={g.n}: oracle ({oracle})")
    if value is None:
        if oracle == "dinic":
            value, side_o, _ = O.dinic(g, cap_now)
        else:
            value, side_o = O.fifo_push_relabel(g, cap_now)
    else:
        side_o = None
    assert v == value, (v, value)
    side, cut = F.min_cut()
    assert cut == value
    if side_o is not None:
        assert np.array_equal(side, side_o)
    if not full:
        return v
    if big:
        log(f"oracle value {value} ({time.time() - t0:.1f}s); layout")
    pg = check_layout(F, g, cap_now)
    cap, cf, e, h, ecap = F.export_state()
    assert np.array_equal(cap, pg.cap)
    assert np.array_equal(ecap, np.asarray(cap_now, dtype=np.int32))
    if big:
        log(f"validator ({time.time() - t0:.1f}s)")
    rc, val, vside, _ = O.validate(pg, cf, e)
    assert rc == 0, f"validator check {rc} failed"
    assert val == value
    assert np.array_equal(vside, side)
    if exact_heights:
        assert np.array_equal(h, O.bfs_heights(pg, cf, e))
    else:
        assert np.array_equal((h >= g.n).astype(np.uint8), vside)
    if big:
        log(f"checked n={g.n} value={v} (oracle+validator {time.time() - t0:.1f}s)")
    return v


def check_edge_flow(F, g, cap_now):
    """mf_edge_flow: every edge within [0, capacity], conservation at every
    vertex but s and t, net flow out of s = value = into t, cut edges
    saturated from the source side and empty from the sink side; the
    handle's own state, value and cut are unchanged."""
    before = F.export_state()
    v = F.value()
    side, _ = F.min_cut()
    flow = F.edge_flow().astype(np.int64)
    cap = np.asarray(cap_now, dtype=np.int64)
    assert flow.shape == (g.m,)
    assert (flow >= 0).all() and (flow <= cap).all()
    tails = g.tails()
    net = np.bincount(g.col, weights=flow, minlength=g.n) - np.bincount(tails, weights=flow, minlength=g.n)
    net = np.rint(net).astype(np.int64)
    inner = np.ones(g.n, dtype=bool)
    inner[[g.s, g.t]] = False
    assert (net[inner] == 0).all()
    assert net[g.t] == v and net[g.s] == -v
    fwd = (side[tails] == 1) & (side[g.col] == 0)
    bwd = (side[tails] == 0) & (side[g.col] == 1)
    assert np.array_equal(flow[fwd], cap[fwd]) and (flow[bwd] == 0).all()
    after = F.export_state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert F.value() == v
    return flow
