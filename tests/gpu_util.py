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


def check_solved(F, g, cap_now, value=None, full=True, oracle="dinic"):
    """Value and canonical cut equal the oracle's; the exported residual state
    passes the validator (and its completion is a valid flow of that value);
    the final heights are the exact global-relabel heights of that state."""
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
    assert np.array_equal(h, O.bfs_heights(pg, cf, e))
    if big:
        log(f"checked n={g.n} value={v} (oracle+validator {time.time() - t0:.1f}s)")
    return v
