"""Pins for the oracle's dynamic route (O4) and for the merged arc-pair layout
and validator (no GPU)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.graphs import tiny_random


def _chain(g, p, batches):
    cap = g.cap.copy()
    for ids, new in batches:
        cap[ids] = new
        v = p.update(ids, new)
        vd, side, _ = O.dinic(g, cap)
        assert v == vd
        assert np.array_equal(p.source_side(), side)
        rc, val, vside, _ = O.validate(p.pg, p.cf, p.e)
        assert rc == 0 and val == vd and np.array_equal(vside, side)
        yield cap, v


@pytest.mark.parametrize("seed", range(150))
def test_tiny_dynamic_chain_matches_recompute(seed):
    g = tiny_random(5000 + seed)
    p = O.PaperSeq(g)
    p.solve()
    rng = np.random.default_rng(seed)
    batches = []
    cap = g.cap.copy()
    for _ in range(4):
        if g.m == 0:
            break
        k = int(rng.integers(1, g.m + 1))
        ids = rng.choice(g.m, k, replace=False).astype(np.int64)
        new = rng.integers(0, 12, k).astype(np.int32)
        batches.append((ids, new))
        cap[ids] = new
    for cap_now, v in _chain(g, p, batches):
        assert v == O.brute_force_min_cut(g, cap_now)[0]


def test_c1_dynamic_chain():
    g = W.c1_random_1k()
    p = O.PaperSeq(g)
    p.solve()
    batches = list(W.batch_chain(g, 0.0125, 5, 100, seed=W.SEED_BASE))
    assert batches[0][0].shape[0] == 100
    for _ in _chain(g, p, batches):
        pass


@pytest.mark.parametrize("kind", ["inc", "dec"])
def test_monotone_and_lipschitz(kind):
    g = W.random_graph(300, 2400, 1, 100, seed=77, s=0, t=299)
    p = O.PaperSeq(g)
    prev = p.solve()
    cap = g.cap.copy()
    rng = np.random.default_rng(9)
    for j in range(6):
        frac = 1.0 if kind == "inc" else 0.0
        ids, new = W.mixed_batch(cap, 120, 100, rng, inc_fraction=frac)
        dcap = int(np.abs(new.astype(np.int64) - cap[ids]).sum())
        cap[ids] = new
        v = p.update(ids, new)
        assert v == O.dinic(g, cap)[0]
        if kind == "inc":
            assert v >= prev
        else:
            assert v <= prev
        assert abs(v - prev) <= dcap
        prev = v


def test_update_step_equals_full_recompute_and_is_order_free():
    """Alg. 5 then the excess recomputation: the resulting state depends only
    on the batch as a set, and matches an incremental booking of the clamps."""
    g = W.random_graph(200, 1600, 1, 50, seed=3, s=0, t=199)
    p = O.PaperSeq(g)
    p.solve()
    rng = np.random.default_rng(4)
    ids, new = W.mixed_batch(g.cap, 300, 50, rng)
    q = O.PaperSeq(g)
    q.cf[:] = p.cf
    q.e[:] = p.e
    perm = rng.permutation(ids.shape[0])
    # incremental booking: clamp only arcs touched by the batch
    pg = p.pg
    cf, e, cap = p.cf.copy(), p.e.copy(), pg.cap.copy()
    tails = pg.tails()
    touched = set()
    for i in range(ids.shape[0]):
        a = pg.edge2arc[ids[i]]
        d = int(new[i]) - int(pg.ecap[ids[i]])
        if a >= 0:
            cf[a] += d
            cap[a] += d
            touched.update([a, pg.twin[a]])
    for a in sorted(touched):
        if cf[a] < 0:
            o = -int(cf[a])
            cf[pg.twin[a]] -= o
            cf[a] = 0
            e[tails[a]] += o
            e[pg.col[a]] -= o
    p.apply_updates(ids, new)
    q.apply_updates(ids[perm], new[perm])
    assert np.array_equal(p.cf, q.cf) and np.array_equal(p.e, q.e)
    # after re-saturation the incremental state matches too
    s = pg.s
    for a in range(pg.row_ptr[s], pg.row_ptr[s + 1]):
        d = int(cf[a])
        if d > 0:
            cf[a] = 0
            cf[pg.twin[a]] += d
            e[pg.col[a]] += d
            e[s] -= d
    assert np.array_equal(cf, p.cf) and np.array_equal(e, p.e)
    assert np.array_equal(cap, p.pg.cap)


# ---------------- merged arc-pair layout ----------------

@pytest.mark.parametrize("seed", range(40))
def test_pair_layout_invariants(seed):
    g = tiny_random(900 + seed, n_hi=12, m_hi=60)
    pg = O.PairGraph.build(g)
    A = pg.A
    tails = pg.tails()
    if A:
        assert np.array_equal(pg.twin[pg.twin], np.arange(A))
        assert np.array_equal(pg.col[pg.twin], tails)
        assert np.all(pg.col != tails)
    # neighbours sorted and distinct inside each list
    for u in range(pg.n):
        nb = pg.col[pg.row_ptr[u]:pg.row_ptr[u + 1]]
        assert np.all(np.diff(nb) > 0)
    # capacities: arc u->v holds the sum over input edges u->v
    etail = g.tails()
    for a in range(A):
        u, v = tails[a], pg.col[a]
        assert pg.cap[a] == g.cap[(etail == u) & (g.col == v)].sum()
    for i in range(g.m):
        a = pg.edge2arc[i]
        if etail[i] == g.col[i]:
            assert a == -1
        else:
            assert tails[a] == etail[i] and pg.col[a] == g.col[i]
    # every unordered pair with an edge appears exactly once per direction
    pairs = {(min(a, b), max(a, b)) for a, b in zip(etail, g.col) if a != b}
    assert A == 2 * len(pairs)


# ---------------- validator rejects planted mistakes ----------------

def _solved_state(seed=11):
    g = W.random_graph(120, 900, 1, 30, seed=seed, s=0, t=119)
    p = O.PaperSeq(g)
    p.solve()
    rc, val, side, flow = O.validate(p.pg, p.cf, p.e)
    assert rc == 0 and val == O.dinic(g)[0]
    return g, p, side


def test_validator_accepts_and_repairs():
    g, p, side = _solved_state()
    rc, val, side2, flow = O.validate(p.pg, p.cf, p.e)
    assert rc == 0
    pg = p.pg
    # repaired pair flow: antisymmetric, within capacity, conserved
    assert np.array_equal(flow, -flow[pg.twin])
    assert np.all(flow <= pg.cap) and np.all(-flow <= pg.cap[pg.twin])
    net = np.zeros(pg.n, dtype=np.int64)
    np.add.at(net, pg.tails(), flow)
    assert net[pg.s] == val and net[pg.t] == -val
    assert np.all(np.delete(net, [pg.s, pg.t]) == 0)


def test_validator_rejects_negative_residual():
    g, p, _ = _solved_state()
    cf = p.cf.copy()
    a = int(np.nonzero(cf > 0)[0][0])
    cf[a] = -1
    assert O.validate(p.pg, cf, p.e)[0] == 1


def test_validator_rejects_broken_pair_sum():
    g, p, _ = _solved_state()
    cf = p.cf.copy()
    a = int(np.nonzero(cf > 0)[0][0])
    cf[a] += 1
    assert O.validate(p.pg, cf, p.e)[0] == 2


def test_validator_rejects_wrong_excess():
    g, p, _ = _solved_state()
    e = p.e.copy()
    e[5] += 1
    assert O.validate(p.pg, p.cf, e)[0] == 3


def test_validator_rejects_unfinished_state():
    g = W.random_graph(120, 900, 1, 30, seed=11, s=0, t=119)
    p = O.PaperSeq(g)
    p.init()
    assert p.loop(max_iter=0) is False
    rc = O.validate(p.pg, p.cf, p.e)[0]
    assert rc in (4, 5)


def test_validator_rejects_dropped_flow():
    """A planted mistake in the oracle's own arithmetic: flow moved along a
    pair without booking the excess is caught."""
    g, p, _ = _solved_state()
    pg = p.pg
    cf = p.cf.copy()
    a = int(np.nonzero(cf > 0)[0][0])
    cf[a] -= 1
    cf[pg.twin[a]] += 1
    assert O.validate(pg, cf, p.e)[0] == 3


@pytest.mark.parametrize("kind", ["inc", "dec"])
def test_biased_families_monotone_and_lipschitz_on_a_grid(kind):
    """The paper's update families with picks biased toward s/t edges: an
    incremental chain never lowers the value, a decremental one never raises
    it, and no batch moves it by more than the capacity it changed."""
    g = W.seg_grid(24, seed=21)
    p = O.PaperSeq(g)
    prev = p.solve()
    cap = g.cap.copy()
    frac = 1.0 if kind == "inc" else 0.0
    for ids, new in W.batch_chain(g, 0.05, 4, 100, seed=31, inc_fraction=frac, p_st=0.5):
        dcap = int(np.abs(new.astype(np.int64) - cap[ids]).sum())
        cap[ids] = new
        v = p.update(ids, new)
        assert v == O.dinic(g, cap)[0]
        assert (v >= prev) if kind == "inc" else (v <= prev)
        assert abs(v - prev) <= dcap
        prev = v
