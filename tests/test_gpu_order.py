"""GPU parity of the vertex numbering: a handle that numbers the vertices by
falling degree (MF_ORDER_DEGREE) takes and returns the caller's vertex and
edge ids, so every exported layout and state, value, cut and height must be
what the oracle computes in the caller's numbering, and what a handle in the
caller's order (MF_ORDER_INPUT) reports."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import check_solved, log
from tests.graphs import from_edges, tiny_random

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


def _hub_graph():
    """An inner hub of about 5000 arcs besides hubs s and t, so that the
    degree order moves every hub to the front."""
    rng = np.random.default_rng(31)
    n = 9000
    hub = 4321
    edges = [(17, v, int(rng.integers(1, 40))) for v in range(0, n, 2) if v != 17]
    edges += [(v, 9000 - 1, int(rng.integers(1, 40))) for v in range(1, n - 1, 3)]
    edges += [(v, hub, int(rng.integers(1, 60))) for v in range(0, n, 4) if v != hub]
    edges += [(hub, v, int(rng.integers(1, 60))) for v in range(2, n, 4) if v != hub]
    edges += [(int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(1, 30))) for _ in range(20000)]
    return from_edges(n, edges, 17, n - 1)


def _graph(which):
    if which == "c1":
        return W.c1_random_1k(), 100, 0.0125
    if which == "grid":
        return W.seg_grid(96, seed=71), 100, 0.01
    if which == "rmat":
        return W.rmat(14, 16, seed=72), 1000, 0.005
    return _hub_graph(), 50, 0.01


@pytest.mark.parametrize("which", ["c1", "grid", "rmat", "hubs"])
def test_degree_order_against_input_order(mf, which):
    """Static solve and a mixed chain of batches on both numberings: equal
    values and canonical cuts, and the renumbered handle's exported layout,
    state and heights pass the oracle's checks in the caller's numbering."""
    g, inc, frac = _graph(which)
    with mf.MaxFlow(g, vertex_order=mf.MF_ORDER_INPUT) as F1, \
            mf.MaxFlow(g, vertex_order=mf.MF_ORDER_DEGREE) as F2:
        assert F1.num_arcs == F2.num_arcs
        v1, v2 = F1.solve(), F2.solve()
        assert v1 == v2
        assert np.array_equal(F1.min_cut()[0], F2.min_cut()[0])
        check_solved(F2, g, g.cap)
        cap = g.cap.copy()
        for j, (ids, new) in enumerate(W.batch_chain(g, frac, 4, inc, seed=W.SEED_BASE + 70)):
            cap[ids] = new
            v1, v2 = F1.update(ids, new), F2.update(ids, new)
            assert v1 == v2, (j, v1, v2)
            assert np.array_equal(F1.min_cut()[0], F2.min_cut()[0])
            check_solved(F2, g, cap)
        # the flow returned per edge is valid for the caller's edges
        f = F2.edge_flow()
        assert np.all(f >= 0) and np.all(f <= cap)
        tails = g.tails()
        net = np.bincount(tails, weights=f, minlength=g.n) - np.bincount(g.col, weights=f, minlength=g.n)
        inner = np.ones(g.n, dtype=bool)
        inner[[g.s, g.t]] = False
        assert np.all(net[inner] == 0)
        assert net[g.s] == F2.value()


@pytest.mark.parametrize("seed", range(3))
def test_repair_bit_exact_through_the_numbering(mf, seed):
    """The batch repair on a renumbered handle, seen through the exported
    state, equals the oracle's sequential repair bit for bit (the exported
    arrays are in the caller's numbering; the local stage is off, since the
    oracle models the paper's repair alone)."""
    g = W.random_graph(600, 4800, 1, 50, seed=300 + seed, s=0, t=599)
    rng = np.random.default_rng(seed)
    with mf.MaxFlow(g, flags=mf.MF_FLAG_GLOBAL_ONLY, vertex_order=mf.MF_ORDER_DEGREE) as F:
        F.solve()
        cap = g.cap.copy()
        for _ in range(3):
            cap0, cf0, e0, _, _ = F.export_state()
            ids, new = W.mixed_batch(cap, int(rng.integers(1, 600)), 50, rng)
            p = O.PaperSeq(g, cap=cap)
            p.cf[:] = cf0
            p.e[:] = e0
            assert np.array_equal(p.pg.cap, cap0)
            p.apply_updates(ids, new)
            cap[ids] = new
            F.set_max_iterations(0)
            try:
                F.update(ids, new)
            except mf.MfError as ex:
                assert ex.code == mf.MF_ETIMEOUT
            capg, cfg, eg, _, ecapg = F.export_state()
            assert np.array_equal(capg, p.pg.cap)
            assert np.array_equal(cfg, p.cf)
            assert np.array_equal(eg, p.e)
            assert np.array_equal(ecapg, cap)
            F.set_max_iterations(-1)
            F.resume()
            check_solved(F, g, cap)


def test_state_moves_between_numberings(mf):
    """A state exported from a renumbered handle imports into a handle in the
    caller's order and into another renumbered one (and back), and all three
    continue a chain of batches to the oracle's values."""
    g = W.rmat(13, 16, seed=73)
    chain = list(W.batch_chain(g, 0.01, 3, 1000, seed=W.SEED_BASE + 74))
    with mf.MaxFlow(g, vertex_order=mf.MF_ORDER_DEGREE) as A, \
            mf.MaxFlow(g, vertex_order=mf.MF_ORDER_INPUT) as B, \
            mf.MaxFlow(g, vertex_order=mf.MF_ORDER_DEGREE) as C:
        A.solve()
        B.solve()
        C.solve()
        cap = g.cap.copy()
        ids, new = chain[0]
        cap[ids] = new
        A.update(ids, new)
        st = A.export_state()
        B.import_state(st[0], st[1], st[2], st[4])
        C.import_state(st[0], st[1], st[2], st[4])
        want = O.dinic(g, cap)[0]
        assert B.resume() == want and C.resume() == want
        # and back: B's state (caller's order, same numbers) into A
        st_b = B.export_state()
        A.import_state(st_b[0], st_b[1], st_b[2], st_b[4])
        assert A.resume() == want
        for ids, new in chain[1:]:
            cap[ids] = new
            want = O.dinic(g, cap)[0]
            assert A.update(ids, new) == want
            assert B.update(ids, new) == want
            assert C.update(ids, new) == want
        check_solved(C, g, cap)


def test_default_order_by_size(mf):
    """MF_ORDER_AUTO keeps the caller's order up to 8192 vertices and numbers
    larger graphs by degree; both report the same results."""
    for g in (W.c1_random_1k(), W.rmat(14, 8, seed=75)):
        with mf.MaxFlow(g) as F, mf.MaxFlow(g, vertex_order=mf.MF_ORDER_INPUT) as G:
            assert F.solve() == G.solve()
            assert np.array_equal(F.min_cut()[0], G.min_cut()[0])
            log(f"n={g.n}: value {F.value()}")
    # tiny graphs with forced degree order, including degenerate ones
    for seed in range(20):
        g = tiny_random(seed, n_hi=14, m_hi=50)
        with mf.MaxFlow(g, vertex_order=mf.MF_ORDER_DEGREE) as F:
            F.solve()
            check_solved(F, g, g.cap)


@pytest.mark.parametrize("order", [1, 2])
def test_local_stage_batches_on_shared_ends(mf, order):
    """Batches drawn from the edges of one inner hub and of s and t: many batch
    ends are the same vertex, so the local pulls' claims contend (a vertex can
    become a giver left in deficit while its own claim as a batch end is still
    pending).  After every batch the value and cut equal the oracle's and the
    exported state passes the validator (no negative residual, excesses and
    deficits routable)."""
    g = _hub_graph()
    tails = g.tails()
    hub = 4321
    near = np.flatnonzero((tails == hub) | (g.col == hub) | (tails == g.s) | (g.col == g.t))
    rng = np.random.default_rng(77 + order)
    with mf.MaxFlow(g, vertex_order=order) as F:
        F.solve()
        cap = g.cap.copy()
        for j in range(6):
            k = int(rng.integers(200, 3000))
            ids = np.sort(rng.choice(near, k, replace=False)).astype(np.int64)
            up = rng.random(k) < 0.5
            new = np.where(up, cap[ids] + rng.integers(1, 80, k), rng.integers(0, cap[ids] + 1)).astype(np.int32)
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)
