"""The seeded generators: determinism and the shapes of the paper-style workloads."""
import hashlib

import numpy as np

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
