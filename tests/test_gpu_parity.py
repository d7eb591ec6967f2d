"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Values must match bit for bit, the canonical minimum cut element by element,
the merged layout and the deterministic steps (initialisation, update repair,
BFS heights) bit for bit; racy sweeps are checked through the validator."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import check_layout, check_solved, log
from tests.graphs import from_edges, tiny_random

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


# ---------------- tiny graphs: every configuration ----------------

@pytest.mark.parametrize("seed", range(120))
def test_tiny_static_and_dynamic(mf, seed):
    g = tiny_random(seed, n_hi=14, m_hi=50)
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap)
        rng = np.random.default_rng(seed)
        cap = g.cap.copy()
        for _ in range(3):
            if g.m == 0:
                break
            k = int(rng.integers(1, g.m + 1))
            ids = rng.choice(g.m, k, replace=False).astype(np.int64)
            new = rng.integers(0, 12, k).astype(np.int32)
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)
            if g.n <= 16:
                assert F.value() == O.brute_force_min_cut(g, cap)[0]


@pytest.mark.parametrize("grid", [1, 2, 8, 64])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("kc", [0, 1, 3, 40])
def test_c1_launch_shapes(mf, grid, mode, kc):
    g = W.c1_random_1k()
    with mf.MaxFlow(g, grid_blocks=grid, mode=mode, kernel_cycles=kc) as F:
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.0125, 3, 100, seed=W.SEED_BASE + 7):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)


def test_c1_chain_against_recompute(mf):
    """Config: 1,000 vertices, 8,000 edges, caps U[1,100]; static then a chain
    of 100-update mixed batches, each checked against a from-scratch oracle."""
    g = W.c1_random_1k()
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.0125, 20, 100, seed=W.SEED_BASE):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)


# ---------------- deterministic steps, bit-exact against the sequential paper route ----------------

def test_init_state_matches_paper_init(mf):
    g = W.random_graph(500, 4000, 0, 60, seed=21, s=3, t=400)
    p = O.PaperSeq(g)
    p.init()
    with mf.MaxFlow(g, max_iterations=0) as F:
        with pytest.raises(mf.MfError) as ei:
            F.solve()
        assert ei.value.code == mf.MF_ETIMEOUT
        cap, cf, e, h, ecap = F.export_state()
        assert np.array_equal(cf, p.cf) and np.array_equal(e, p.e)
        # the global relabel of the first round ran; its heights are exact
        assert np.array_equal(h, O.bfs_heights(p.pg, p.cf, p.e))
        F.set_max_iterations(-1)
        F.resume()
        check_solved(F, g, g.cap)


@pytest.mark.parametrize("seed", range(6))
def test_update_repair_matches_paper_updates(mf, seed):
    """The state after the batch repair (Alg. 5 with the re-saturation of
    Alg. 4) equals the oracle's sequential repair bit for bit; the local stage
    is off, since the oracle models the paper's repair alone."""
    g = W.random_graph(400, 3200, 1, 50, seed=100 + seed, s=0, t=399)
    rng = np.random.default_rng(seed)
    with mf.MaxFlow(g, flags=mf.MF_FLAG_GLOBAL_ONLY) as F:
        F.solve()
        cap = g.cap.copy()
        for j in range(3):
            cap0, cf0, e0, _, ecap0 = F.export_state()
            ids, new = W.mixed_batch(cap, int(rng.integers(1, 400)), 50, rng)
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
            capg, cfg, eg, hg, ecapg = F.export_state()
            assert np.array_equal(capg, p.pg.cap)
            assert np.array_equal(cfg, p.cf)
            assert np.array_equal(eg, p.e)
            assert np.array_equal(ecapg, cap)
            F.set_max_iterations(-1)
            F.resume()
            check_solved(F, g, cap)


@pytest.mark.parametrize("p_st", [0.0, 0.3])
@pytest.mark.parametrize("which", ["c1", "grid", "rmat"])
def test_local_stage_against_global_only(mf, which, p_st):
    """Dynamic updates with the local stage (default) and without it
    (MF_FLAG_GLOBAL_ONLY) reach the same value and canonical cut as the
    oracle after every batch of a mixed chain, including batches biased to
    the edges at s and t (which cross the cut)."""
    if which == "c1":
        g, inc, frac = W.c1_random_1k(), 100, 0.0125
    elif which == "grid":
        g, inc, frac = W.seg_grid(128, seed=61), 100, 0.01
    else:
        g, inc, frac = W.rmat(15, 16, seed=62), 1000, 0.002
    with mf.MaxFlow(g) as L, mf.MaxFlow(g, flags=mf.MF_FLAG_GLOBAL_ONLY) as G:
        assert L.solve() == G.solve()
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, frac, 5, inc, seed=W.SEED_BASE + 60, p_st=p_st):
            cap[ids] = new
            vl = L.update(ids, new)
            assert vl == G.update(ids, new)
            assert np.array_equal(L.min_cut()[0], G.min_cut()[0])
            check_solved(L, g, cap)


def test_clamp_with_parallel_and_antiparallel_edges(mf):
    """Several updates land on one arc pair (duplicates and the reverse
    direction) in the same batch; the clamp must act once on the summed delta."""
    edges = [(0, 1, 50), (1, 2, 30), (1, 2, 20), (2, 1, 5), (2, 3, 60), (1, 3, 10), (3, 2, 4)]
    g = from_edges(4, edges, 0, 3)
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        tails = g.tails()
        sel = np.nonzero(((tails == 1) & (g.col == 2)) | ((tails == 2) & (g.col == 1)))[0]
        ids = sel.astype(np.int64)
        new = np.zeros(ids.shape[0], dtype=np.int32)
        cap[ids] = new
        F.update(ids, new)
        check_solved(F, g, cap)


# ---------------- paper-scale workloads ----------------

def test_c2_grid_static_and_batches(mf):
    """Config: 512x512 segmentation grid, 1% mixed batches."""
    g = W.c2_grid_512()
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap, oracle="fifo")
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.01, 2, 100, seed=W.SEED_BASE + 1):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, oracle="fifo")


def test_c3_rmat_static_and_batch(mf):
    """Config: R-MAT scale 20, 0.1%, 1% and 10% mixed batches (full parity at
    the full size: value, cut, validator, heights)."""
    g = W.c3_rmat20()
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap, oracle="fifo")
        cap = g.cap.copy()
        for frac in (0.001, 0.01, 0.1):
            ids, new = W.mixed_batch(cap, W.batch_size(g.m, frac), 1000,
                                     W.rng_for(W.SEED_BASE + 2, 9, int(frac * 1e4)))
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, oracle="fifo")


def _certify_at_any_size(F, g, rp, col, twin):
    """The validator's local checks in vectorised form (no max-flow route):
    c_f >= 0, pair sums, every excess equals its residual in-minus-out change,
    positive excess only on the source side and deficits only on the sink side
    of the canonical cut, no residual arc from the source side to the sink
    side, and a cut capacity equal to the value."""
    cap, cf, e, _, _ = F.export_state()
    value = F.value()
    side, cut = F.min_cut()
    assert cut == value
    assert (cf >= 0).all()
    assert np.array_equal(cap.astype(np.int64) + cap[twin], cf.astype(np.int64) + cf[twin])
    tails = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(rp))
    booked = np.bincount(tails, weights=(cf.astype(np.int64) - cap).astype(np.float64), minlength=g.n)
    assert np.array_equal(booked.astype(np.int64), e)
    inner = np.ones(g.n, dtype=bool)
    inner[[g.s, g.t]] = False
    assert (side[(e > 0) & inner] == 1).all() and (side[(e < 0) & inner] == 0).all()
    assert side[g.s] == 1 and side[g.t] == 0
    crossing = (side[tails] == 1) & (side[col] == 0)
    assert not (cf[crossing] > 0).any()
    assert value == int(e[g.t]) + int(e[inner & (e < 0)].sum())
    return value


@pytest.mark.timeout(900)
def test_c5_full_size_against_oracle(mf):
    """Config: the served R-MAT scale 22 graph (4,194,304 V, 67,108,864 E) at
    full size.  The static solve and the first request of the served stream
    (10 to 100k edges, log-uniform) are checked in full against the oracle:
    value and canonical cut against the FIFO push-relabel (O2), merged layout,
    and the exported state through the whole validator, including its
    phase-two routes that return every excess to s and fill every deficit
    from t.  The next two requests are checked for dynamic == a fresh static
    solve of the same capacities and by the validator's local checks
    (_certify_at_any_size)."""
    g = W.c5_rmat22()
    log(f"c5 graph built: n={g.n} m={g.m}")
    with mf.MaxFlow(g) as D, mf.MaxFlow(g) as S:
        rp, col, twin, _ = D.export_graph()
        v = D.solve()
        assert S.solve() == v
        check_solved(D, g, g.cap, oracle="fifo")
        cap = g.cap.copy()
        for j, (ids, new) in enumerate(W.request_stream(g, 3, W.SEED_BASE + 4)):
            cap[ids] = new
            v = D.update(ids, new)
            S.set_capacities(ids, new)
            assert S.solve() == v, j
            if j == 0:
                check_solved(D, g, cap, oracle="fifo")
            else:
                assert _certify_at_any_size(D, g, rp, col, twin) == v
            log(f"c5 request {j}: {ids.shape[0]} edges, value {v}")


# ---------------- static comparator path ----------------

def test_set_capacities_then_static_equals_dynamic(mf):
    g = W.random_graph(2000, 16000, 1, 100, seed=5, s=0, t=1999)
    ids, new = W.mixed_batch(g.cap, 500, 100, np.random.default_rng(1))
    cap = W.apply_batch(g.cap, ids, new)
    with mf.MaxFlow(g) as D, mf.MaxFlow(g) as S:
        D.solve()
        vd = D.update(ids, new)
        S.set_capacities(ids, new)
        with pytest.raises(mf.MfError) as ei:
            S.value()
        assert ei.value.code == mf.MF_ESTATE
        vs = S.solve()
        assert vd == vs == O.dinic(g, cap)[0]
        assert np.array_equal(D.min_cut()[0], S.min_cut()[0])


def test_device_batch_from_torch(mf):
    import torch
    g = W.c1_random_1k()
    ids, new = next(W.batch_chain(g, 0.0125, 1, 100, seed=3))
    cap = W.apply_batch(g.cap, ids, new)
    with mf.MaxFlow(g) as F:
        F.solve()
        di = torch.from_numpy(ids).to("cuda")
        dc = torch.from_numpy(new).to("cuda")
        torch.cuda.synchronize()
        F.update_device(di, dc)
        check_solved(F, g, cap)


# ---------------- error paths ----------------

def test_errors_leave_the_handle_unchanged(mf):
    g = W.c1_random_1k()
    with mf.MaxFlow(g) as F:
        with pytest.raises(mf.MfError) as ei:
            F.update(np.array([0], np.int64), np.array([1], np.int32))
        assert ei.value.code == mf.MF_ESTATE
        v = F.solve()
        before = F.export_state()
        bad = [
            (np.array([3, 3], np.int64), np.array([1, 2], np.int32)),       # duplicate
            (np.array([g.m], np.int64), np.array([1], np.int32)),           # id range
            (np.array([-1], np.int64), np.array([1], np.int32)),            # id range
            (np.array([5], np.int64), np.array([-4], np.int32)),            # negative
            (np.array([5], np.int64), np.array([F.cap_limit + 1], np.int32)),
        ]
        for ids, new in bad:
            with pytest.raises(mf.MfError) as ei:
                F.update(ids, new)
            assert ei.value.code == mf.MF_EINVAL
            after = F.export_state()
            for a, b in zip(before, after):
                assert np.array_equal(a, b)
            assert F.value() == v
        # an empty batch is a no-op
        assert F.update(np.zeros(0, np.int64), np.zeros(0, np.int32)) == v


def test_iteration_limit_and_resume(mf):
    g = W.seg_grid(64, seed=3)
    with mf.MaxFlow(g, max_iterations=1) as F:
        with pytest.raises(mf.MfError) as ei:
            F.solve()
        assert ei.value.code == mf.MF_ETIMEOUT
        with pytest.raises(mf.MfError):
            F.value()
        F.set_max_iterations(-1)
        F.resume()
        check_solved(F, g, g.cap)


# ---------------- degenerate graphs ----------------

@pytest.mark.parametrize("case", ["no_out_of_s", "t_unreachable", "zero_caps", "only_loops",
                                  "direct_edge", "two_vertices_empty"])
def test_degenerate(mf, case):
    if case == "no_out_of_s":
        g = from_edges(4, [(1, 2, 5), (2, 3, 5)], 0, 3)
    elif case == "t_unreachable":
        g = from_edges(4, [(0, 1, 5), (1, 2, 5)], 0, 3)
    elif case == "zero_caps":
        g = from_edges(4, [(0, 1, 0), (1, 3, 0), (0, 3, 0)], 0, 3)
    elif case == "only_loops":
        g = from_edges(3, [(0, 0, 5), (1, 1, 5), (2, 2, 7)], 0, 2)
    elif case == "direct_edge":
        g = from_edges(2, [(0, 1, 9), (0, 1, 4), (1, 0, 3)], 0, 1)
    else:
        g = from_edges(2, [], 0, 1)
    with mf.MaxFlow(g) as F:
        F.solve()
        check_solved(F, g, g.cap)
        if g.m:
            ids = np.arange(g.m, dtype=np.int64)
            new = (np.arange(g.m) % 3 + 1).astype(np.int32)
            F.update(ids, new)
            cap = g.cap.copy()
            cap[ids] = new
            check_solved(F, g, cap)


def test_hubs_long_lists(mf):
    """Vertices with lists longer than one lane's share and than one BFS item
    (hub s, hub t and an inner hub of degree 3000)."""
    rng = np.random.default_rng(8)
    n = 4000
    hub = 7
    edges = [(0, v, int(rng.integers(1, 50))) for v in range(2, n)]
    edges += [(v, 1, int(rng.integers(1, 50))) for v in range(2, n, 2)]
    edges += [(v, hub, int(rng.integers(1, 50))) for v in range(3, n, 2)]
    edges += [(hub, v, int(rng.integers(1, 50))) for v in range(2, n, 4)]
    g = from_edges(n, edges, 0, 1)
    for grid in (1, 16):
        with mf.MaxFlow(g, grid_blocks=grid) as F:
            F.solve()
            check_solved(F, g, g.cap)
            ids, new = W.mixed_batch(g.cap, 2000, 50, np.random.default_rng(grid))
            cap = W.apply_batch(g.cap, ids, new)
            F.update(ids, new)
            check_solved(F, g, cap)


def test_huge_hubs_visited_by_workgroups(mf):
    """Two inner hubs with about 7000 arcs each (above the workgroup-visit
    threshold of 4096) besides hub s and hub t: static solve and an update,
    with one workgroup, a cooperative grid, topology mode, and inside a batch
    with 256- and 1024-thread workgroups."""
    rng = np.random.default_rng(12)
    n = 14000
    h1, h2 = 5, 6
    edges = [(0, v, int(rng.integers(1, 40))) for v in range(7, n)]
    edges += [(v, 1, int(rng.integers(1, 40))) for v in range(7, n, 3)]
    edges += [(v, h1, int(rng.integers(1, 60))) for v in range(8, n, 3)]
    edges += [(h1, v, int(rng.integers(1, 60))) for v in range(9, n, 3)]
    edges += [(v, h2, int(rng.integers(1, 60))) for v in range(9, n, 3)]
    edges += [(h2, v, int(rng.integers(1, 60))) for v in range(7, n, 3)]
    edges += [(h1, h2, 500), (h2, h1, 500)]
    g = from_edges(n, edges, 0, 1)
    deg = np.diff(g.row_ptr) + np.bincount(g.col, minlength=n)
    assert deg[h1] > 4096 and deg[h2] > 4096
    cap2 = None
    for grid, mode in ((1, 0), (16, 0), (16, 1)):
        with mf.MaxFlow(g, grid_blocks=grid, mode=mode) as F:
            F.solve()
            check_solved(F, g, g.cap)
            ids, new = W.mixed_batch(g.cap, 3000, 50, np.random.default_rng(grid + mode))
            cap2 = W.apply_batch(g.cap, ids, new)
            F.update(ids, new)
            check_solved(F, g, cap2)
    for block in (256, 1024):
        with mf.Batch([g, g], caps=[g.cap, cap2], n_classes=1, block=[block] * 4) as B:
            vals = B.solve()
            assert vals[0] == O.dinic(g, g.cap)[0] and vals[1] == O.dinic(g, cap2)[0]


@pytest.mark.parametrize("kind", ["inc", "dec", "mixed"])
@pytest.mark.parametrize("which", ["grid", "rmat"])
def test_update_families_with_st_bias(mf, kind, which):
    """The paper's incremental, decremental and mixed update families, with
    batch edges drawn from the edges out of s and into t with probability
    0.3: every update matches the oracle (value, cut, validated state, exact
    heights), incremental chains never lower the value and decremental ones
    never raise it."""
    g = W.seg_grid(128, seed=31) if which == "grid" else W.rmat(15, 16, seed=32)
    frac = {"inc": 1.0, "dec": 0.0, "mixed": 0.5}[kind]
    inc = 100 if which == "grid" else 1000
    with mf.MaxFlow(g) as F:
        prev = F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.02, 3, inc, seed=W.SEED_BASE + 33, inc_fraction=frac, p_st=0.3):
            cap[ids] = new
            v = F.update(ids, new)
            check_solved(F, g, cap)
            if kind == "inc":
                assert v >= prev
            elif kind == "dec":
                assert v <= prev
            prev = v


@pytest.mark.parametrize("solo", [-1, 1, 128, 1 << 20])
def test_small_bfs_frontiers_on_one_workgroup(mf, solo):
    """BFS levels whose frontier holds at most `solo_items` items run on the
    first workgroup alone (-1: never; 1: single-item levels; 2^20: every
    level).  Values, cuts, validated states and the exact final heights stay
    the same, for a static solve and updates."""
    g = W.seg_grid(128, seed=12)
    with mf.MaxFlow(g, grid_blocks=8, solo_items=solo) as F:
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.01, 2, 100, seed=W.SEED_BASE + 12):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)


def test_repeat_runs_identical_value_and_cut(mf):
    g = W.seg_grid(128, seed=11)
    value, side, _ = O.dinic(g)
    for rep in range(4):
        with mf.MaxFlow(g, grid_blocks=[0, 4, 32, 1][rep]) as F:
            assert F.solve() == value
            assert np.array_equal(F.min_cut()[0], side)


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("which", ["grid", "rmat"])
def test_gap_heuristic_on_and_off(mf, flags, which):
    """The gap heuristic only changes the schedule: values, cuts and the
    validated state are the same with it on (default) and off."""
    g = W.seg_grid(96, seed=4) if which == "grid" else W.rmat(14, 16, seed=6)
    inc = 100 if which == "grid" else 1000
    with mf.MaxFlow(g, flags=flags) as F:
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.01, 3, inc, seed=W.SEED_BASE + 11):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap)
