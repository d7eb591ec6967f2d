"""The seeded generators: determinism and the shapes of the paper-style workloads."""
import hashlib

import numpy as np
import pytest

import workloads as W


def _digest(g):
    h = hashlib.sha256()
    for a in (g.row_ptr, g.col, g.cap):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(f"{g.n},{g.s},{g.t}".encode())
    return h.hexdigest()


def test_deterministic():
    assert _digest(W.c1_random_1k()) == _digest(W.c1_random_1k())
    assert _digest(W.seg_grid(32, 7)) == _digest(W.seg_grid(32, 7))
    assert _digest(W.rmat(10, 16, 7)) == _digest(W.rmat(10, 16, 7))
    assert _digest(W.rmat(10, 16, 7)) != _digest(W.rmat(10, 16, 8))


def test_c1_shape():
    g = W.c1_random_1k()
    assert (g.n, g.m, g.s, g.t) == (1000, 8000, 0, 999)
    assert g.cap.min() >= 1 and g.cap.max() <= 100
    assert np.all(g.tails() != g.col)
    assert np.all(np.diff(g.row_ptr) >= 0) and g.row_ptr[-1] == g.m


def test_grid_shape():
    side = 64
    g = W.seg_grid(side, 1)
    npx = side * side
    assert g.n == npx + 2 and (g.s, g.t) == (npx, npx + 1)
    assert g.m == 4 * side * (side - 1) + 2 * npx
    tails = g.tails()
    nl = (tails < npx) & (g.col < npx)
    assert g.cap[nl].min() >= 1 and g.cap[nl].max() <= 101
    tl = ~nl
    assert g.cap[tl].min() >= 0 and g.cap[tl].max() <= 200
    # both directions of an n-link share one capacity
    key = dict(zip(zip(tails[nl].tolist(), g.col[nl].tolist()), g.cap[nl].tolist()))
    assert all(key[(v, u)] == c for (u, v), c in key.items())
    # 4-connectivity
    dx = np.abs(tails[nl] % side - g.col[nl] % side) + np.abs(tails[nl] // side - g.col[nl] // side)
    assert np.all(dx == 1)


def test_rmat_shape():
    g = W.rmat(12, 16, 3)
    assert g.n == 4096 and g.m == 16 * 4096
    assert np.all(g.tails() != g.col)
    deg = np.bincount(g.tails(), minlength=g.n) + np.bincount(g.col, minlength=g.n)
    order = np.lexsort((np.arange(g.n), -deg))
    assert (g.s, g.t) == (int(order[0]), int(order[1]))
    assert g.cap.min() >= 1 and g.cap.max() <= 1000
    # heavy tail: the top vertex is far above the mean degree
    assert deg.max() > 20 * deg.mean()


def test_batches():
    g = W.c1_random_1k()
    chain = list(W.batch_chain(g, 0.0125, 3, 100, seed=5))
    cap = g.cap.copy()
    for ids, new in chain:
        assert ids.shape == (100,) and np.unique(ids).shape == (100,)
        old = cap[ids].astype(np.int64)
        assert np.all(new[:50] > old[:50]) and np.all(new[:50] <= old[:50] + 100)
        assert np.all(new[50:] <= old[50:]) and np.all(new[50:] >= 0)
        cap[ids] = new
    assert W.batch_size(1570816, 0.01) == 15708


# ---------------- update families and the s/t bias ----------------

def test_st_edges_are_the_edges_out_of_s_and_into_t():
    g = W.seg_grid(16, seed=3)
    tails = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    st = W.st_edges(g)
    want = [i for i in range(g.m) if tails[i] == g.s or g.col[i] == g.t]
    assert st.tolist() == want
    assert st.shape[0] == 2 * 16 * 16  # one t-link each way per pixel


@pytest.mark.parametrize("p_st", [0.0, 0.3, 1.0])
def test_biased_picks_are_distinct_and_seeded(p_st):
    g = W.seg_grid(32, seed=5)
    st = W.st_edges(g)
    a = W.pick_edges(g.m, 500, np.random.default_rng(7), st, p_st)
    b = W.pick_edges(g.m, 500, np.random.default_rng(7), st, p_st)
    assert np.array_equal(a, b)
    assert np.unique(a).shape[0] == 500 and a.min() >= 0 and a.max() < g.m
    share = np.isin(a, st).mean()
    if p_st == 1.0:
        assert share == 1.0
    elif p_st == 0.0:
        # unbiased: the s/t share is about their share of all edges (2048 of 6016)
        assert abs(share - st.shape[0] / g.m) < 0.1
    else:
        assert abs(share - p_st) < 0.1


def test_bias_capped_by_the_available_edges():
    g = W.c1_random_1k()
    st = W.st_edges(g)
    ids = W.pick_edges(g.m, 100, np.random.default_rng(1), st, 1.0)
    assert np.unique(ids).shape[0] == 100
    assert np.isin(ids, st).sum() == st.shape[0]  # every s/t edge, the rest elsewhere


def test_unbiased_chain_unchanged_by_the_knob():
    g = W.c1_random_1k()
    a = list(W.batch_chain(g, 0.0125, 3, 100, seed=11))
    b = list(W.batch_chain(g, 0.0125, 3, 100, seed=11, p_st=0.0))
    for (i0, n0), (i1, n1) in zip(a, b):
        assert np.array_equal(i0, i1) and np.array_equal(n0, n1)


@pytest.mark.parametrize("inc_fraction", [1.0, 0.0])
def test_update_families_move_capacities_one_way(inc_fraction):
    g = W.seg_grid(24, seed=9)
    cur = g.cap.copy()
    for ids, new in W.batch_chain(g, 0.05, 3, 100, seed=13, inc_fraction=inc_fraction, p_st=0.5):
        old = cur[ids]
        if inc_fraction == 1.0:
            assert (new > old).all()
        else:
            assert (new <= old).all() and (new >= 0).all()
        cur[ids] = new
