"""Pins for the CPU oracle (no GPU): brute force, closed forms, a library
max-flow routine, textbook fixtures and the max-flow / min-cut invariants."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import maximum_bipartite_matching, maximum_flow

import oracle as O
import workloads as W
from tests.graphs import from_edges, read_golden, tiny_random


def _flow_is_valid(g, flow, value, cap=None):
    cap = g.cap if cap is None else cap
    assert np.all(flow >= 0) and np.all(flow <= cap)
    net = np.zeros(g.n, dtype=np.int64)
    tails = g.tails()
    np.add.at(net, tails, -flow)
    np.add.at(net, g.col, flow)
    for v in range(g.n):
        if v == g.s:
            assert net[v] == -value
        elif v == g.t:
            assert net[v] == value
        else:
            assert net[v] == 0


def _cut_capacity(g, side, cap=None):
    cap = g.cap if cap is None else cap
    tails = g.tails()
    return int(cap[(side[tails] == 1) & (side[g.col] == 0)].sum())


def _scipy_value(g, cap=None):
    cap = g.cap if cap is None else cap
    keep = g.tails() != g.col  # scipy rejects nothing, but self-loops carry no flow
    M = csr_matrix((cap[keep].astype(np.int32), (g.tails()[keep], g.col[keep])), shape=(g.n, g.n))
    return int(maximum_flow(M, g.s, g.t, method="dinic").flow_value)


@pytest.mark.parametrize("seed", range(400))
def test_routes_agree_with_brute_force(seed):
    g = tiny_random(seed)
    vb, union = O.brute_force_min_cut(g)
    v1, side1, flow1 = O.dinic(g)
    v2, side2 = O.fifo_push_relabel(g)
    p = O.PaperSeq(g)
    v4 = p.solve()
    assert v1 == vb == v2 == v4
    # canonical cut = union of all minimising source sides
    assert np.array_equal(side1, union)
    assert np.array_equal(side2, union)
    assert np.array_equal(p.source_side(), union)
    _flow_is_valid(g, flow1, v1)
    assert _cut_capacity(g, side1) == v1


@pytest.mark.parametrize("seed", range(30))
def test_dinic_matches_library_maxflow(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(20, 400))
    m = int(rng.integers(n, 8 * n))
    g = W.random_graph(n, m, 0, 1000, seed=seed, s=0, t=n - 1)
    v1, side, flow = O.dinic(g)
    assert v1 == _scipy_value(g)
    _flow_is_valid(g, flow, v1)
    assert _cut_capacity(g, side) == v1


def test_c1_workload_all_routes():
    g = W.c1_random_1k()
    v1, s1, f1 = O.dinic(g)
    v2, s2 = O.fifo_push_relabel(g)
    p = O.PaperSeq(g)
    assert v1 == v2 == p.solve() == _scipy_value(g)
    assert np.array_equal(s1, s2) and np.array_equal(s1, p.source_side())
    _flow_is_valid(g, f1, v1)


def test_golden_textbook_network():
    g, steps = read_golden("clrs_flow_network.txt")
    (_, value), = steps
    assert O.dinic(g)[0] == value
    assert O.fifo_push_relabel(g)[0] == value
    assert O.brute_force_min_cut(g)[0] == value
    assert O.PaperSeq(g).solve() == value


def test_golden_dynamic_diamond():
    g, steps = read_golden("diamond_dynamic.txt")
    p = O.PaperSeq(g)
    assert steps[0][0] is None
    assert p.solve() == steps[0][1]
    cap = g.cap.copy()
    for (ids, new), value in steps[1:]:
        cap[ids] = new
        assert p.update(ids, new) == value
        assert O.dinic(g, cap)[0] == value
        assert O.brute_force_min_cut(g, cap)[0] == value


# ---------------- closed forms ----------------

@pytest.mark.parametrize("seed", range(10))
def test_path_is_min_capacity(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 30))
    caps = rng.integers(0, 100, k + 1)
    n = k + 2
    edges = [(i, i + 1, int(caps[i])) for i in range(k + 1)]
    g = from_edges(n, edges, 0, n - 1)
    assert O.dinic(g)[0] == O.fifo_push_relabel(g)[0] == O.PaperSeq(g).solve() == int(caps.min())


@pytest.mark.parametrize("seed", range(10))
def test_disjoint_paths_sum_of_minima(seed):
    rng = np.random.default_rng(100 + seed)
    npaths = int(rng.integers(1, 8))
    n, edges, expect = 2, [], 0
    for _ in range(npaths):
        ln = int(rng.integers(1, 6))
        caps = rng.integers(1, 50, ln + 1)
        verts = [0] + list(range(n, n + ln)) + [1]
        n += ln
        edges += [(verts[i], verts[i + 1], int(caps[i])) for i in range(ln + 1)]
        expect += int(caps.min())
    g = from_edges(n, edges, 0, 1)
    assert O.dinic(g)[0] == O.fifo_push_relabel(g)[0] == O.PaperSeq(g).solve() == expect


@pytest.mark.parametrize("seed", range(10))
def test_star_sum_of_min(seed):
    rng = np.random.default_rng(200 + seed)
    k = int(rng.integers(1, 50))
    cs, ct = rng.integers(0, 100, k), rng.integers(0, 100, k)
    edges = [(0, 2 + i, int(cs[i])) for i in range(k)] + [(2 + i, 1, int(ct[i])) for i in range(k)]
    g = from_edges(k + 2, edges, 0, 1)
    expect = int(np.minimum(cs, ct).sum())
    assert O.dinic(g)[0] == O.fifo_push_relabel(g)[0] == O.PaperSeq(g).solve() == expect


def test_grid_without_nlinks_is_sum_of_tlink_minima():
    g = W.seg_grid(24, seed=5)
    npx = 24 * 24
    cap = g.cap.copy()
    tails = g.tails()
    nlink = (tails < npx) & (g.col < npx)
    cap[nlink] = 0
    sp = np.zeros(npx, dtype=np.int64)
    pt = np.zeros(npx, dtype=np.int64)
    src_mask = tails == g.s
    sp[g.col[src_mask]] = cap[src_mask]
    snk_mask = g.col == g.t
    pt[tails[snk_mask]] = cap[snk_mask]
    expect = int(np.minimum(sp, pt).sum())
    assert O.dinic(g, cap)[0] == O.fifo_push_relabel(g, cap)[0] == expect
    assert O.PaperSeq(g, cap=cap).solve() == expect


def test_no_path_is_zero():
    g = from_edges(5, [(0, 1, 5), (1, 2, 5), (3, 4, 9), (4, 3, 9)], 0, 4)
    v, side, _ = O.dinic(g)
    assert v == 0 and O.fifo_push_relabel(g)[0] == 0 and O.PaperSeq(g).solve() == 0
    # nothing reaches t except 3: canonical source side is everything else
    assert side.tolist() == [1, 1, 1, 0, 0]


def test_complete_digraph_unit_caps():
    n = 9
    edges = [(u, v, 1) for u in range(n) for v in range(n) if u != v]
    g = from_edges(n, edges, 0, n - 1)
    assert O.dinic(g)[0] == O.fifo_push_relabel(g)[0] == O.PaperSeq(g).solve() == n - 1


@pytest.mark.parametrize("seed", range(10))
def test_unit_bipartite_is_max_matching(seed):
    rng = np.random.default_rng(300 + seed)
    L, R = int(rng.integers(1, 30)), int(rng.integers(1, 30))
    adj = rng.random((L, R)) < 0.15
    s, t = L + R, L + R + 1
    edges = [(s, i, 1) for i in range(L)] + [(L + j, t, 1) for j in range(R)]
    edges += [(i, L + j, 1) for i in range(L) for j in range(R) if adj[i, j]]
    g = from_edges(L + R + 2, edges, s, t)
    match = maximum_bipartite_matching(csr_matrix(adj.astype(np.int32)), perm_type="column")
    expect = int((match >= 0).sum())
    assert O.dinic(g)[0] == O.fifo_push_relabel(g)[0] == O.PaperSeq(g).solve() == expect


# ---------------- BFS heights against a library shortest-path routine ----------------

@pytest.mark.parametrize("seed", range(20))
def test_bfs_heights_match_library_shortest_paths(seed):
    from scipy.sparse.csgraph import shortest_path
    g = W.random_graph(60, 240, 0, 20, seed=seed, s=0, t=59)
    p = O.PaperSeq(g)
    p.init()
    p.loop(max_iter=int(seed % 4))   # a mid-run state, deficits possible
    pg = p.pg
    h = O.bfs_heights(pg, p.cf, p.e)
    n = pg.n
    roots = [v for v in range(n) if v == pg.t or (v != pg.s and p.e[v] < 0)]
    # reversed residual graph: w -> v for residual v -> w; a super root n -> roots;
    # nothing may enter s
    tails = pg.tails()
    keep = (p.cf > 0) & (tails != pg.s)
    rows = np.concatenate([pg.col[keep], np.full(len(roots), n)])
    cols = np.concatenate([tails[keep], np.array(roots, dtype=np.int64)])
    M = csr_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n + 1, n + 1))
    d = shortest_path(M, directed=True, unweighted=True, indices=n)[:n]
    expect = np.where(np.isinf(d), n, d - 1).astype(np.int64)
    expect[pg.s] = n
    assert np.array_equal(h.astype(np.int64), expect)


def _relabel(g, new_of_old):
    """g with vertex v renamed new_of_old[v] (edge i keeps its capacity and
    becomes edge eid[i] of the relabelled CSR)."""
    tails = g.tails()
    nt = new_of_old[tails].astype(np.int64)
    nh = new_of_old[g.col].astype(np.int64)
    order = np.argsort((nt << 32) | nh, kind="stable")
    eid = np.empty(g.m, dtype=np.int64)
    eid[order] = np.arange(g.m)
    row_ptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(nt, minlength=g.n), out=row_ptr[1:])
    h = W.Graph(g.n, row_ptr, nh[order].astype(np.int32), g.cap[order].copy(), int(new_of_old[g.s]),
                int(new_of_old[g.t]))
    return h, eid


@pytest.mark.parametrize("seed", range(40))
def test_relabelling_maps_value_cut_and_heights(seed):
    """A handle may number the vertices in another order inside (by falling
    degree, say) and map its results back: what makes that exact is that a
    relabelling leaves the maximum-flow value unchanged and maps the canonical
    cut (the vertices that cannot reach t in the residual graph) and the exact
    BFS heights through the permutation.  Checked with Dinic on random graphs
    (parallel and antiparallel edges, self-loops), under the degree order the
    device build uses and under random orders, before and after a batch."""
    rng = np.random.default_rng(seed)
    g = tiny_random(seed, n_hi=30, m_hi=120)
    deg = np.diff(g.row_ptr) + np.bincount(g.col, minlength=g.n)
    orders = [np.argsort(-deg, kind="stable"), rng.permutation(g.n)]
    v0, side0, _ = O.dinic(g, g.cap)
    ids = rng.choice(g.m, max(1, g.m // 4), replace=False).astype(np.int64) if g.m else np.zeros(0, np.int64)
    new = rng.integers(0, 15, ids.shape[0]).astype(np.int32)
    cap1 = g.cap.copy()
    cap1[ids] = new
    v1, side1, _ = O.dinic(g, cap1)
    pg = O.PairGraph.build(g, g.cap)
    for order in orders:
        new_of_old = np.empty(g.n, dtype=np.int64)
        new_of_old[order] = np.arange(g.n)
        h, eid = _relabel(g, new_of_old)
        w0, hside0, _ = O.dinic(h, h.cap)
        assert w0 == v0
        assert np.array_equal(hside0[new_of_old], side0)
        hcap1 = h.cap.copy()
        hcap1[eid[ids]] = new
        w1, hside1, _ = O.dinic(h, hcap1)
        assert w1 == v1
        assert np.array_equal(hside1[new_of_old], side1)
        # exact global-relabel heights of the initial residual state map the same way
        hp = O.PairGraph.build(h, h.cap)
        e0 = np.zeros(g.n, dtype=np.int64)
        assert np.array_equal(O.bfs_heights(hp, hp.cap.copy(), e0)[new_of_old],
                              O.bfs_heights(pg, pg.cap.copy(), e0))
