"""GPU parity of the valid-flow extraction (mf_edge_flow) and of the Dynamic
Push-Pull update (MF_FLAG_PUSH_PULL) against the CPU oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import check_edge_flow, check_solved, log
from tests.graphs import from_edges, tiny_random

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


# ---------------- valid flow per edge ----------------

@pytest.mark.parametrize("seed", range(40))
def test_edge_flow_tiny(mf, seed):
    g = tiny_random(seed, n_hi=14, m_hi=50)
    with mf.MaxFlow(g) as F:
        F.solve()
        check_edge_flow(F, g, g.cap)
        rng = np.random.default_rng(seed)
        cap = g.cap.copy()
        for _ in range(2):
            if g.m == 0:
                break
            k = int(rng.integers(1, g.m + 1))
            ids = rng.choice(g.m, k, replace=False).astype(np.int64)
            new = rng.integers(0, 12, k).astype(np.int32)
            cap[ids] = new
            F.update(ids, new)
            check_edge_flow(F, g, cap)
            check_solved(F, g, cap)


@pytest.mark.parametrize("grid", [1, 8])
def test_edge_flow_c1(mf, grid):
    g = W.c1_random_1k()
    with mf.MaxFlow(g, grid_blocks=grid) as F:
        F.solve()
        check_edge_flow(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.0125, 3, 100, seed=W.SEED_BASE + 41):
            cap[ids] = new
            F.update(ids, new)
            check_edge_flow(F, g, cap)
            # the extraction left the handle's state alone: the chain goes on exactly
            check_solved(F, g, cap)


def test_edge_flow_parallel_edges(mf):
    """Duplicate and antiparallel edges share one arc pair; the pair's flow is
    split among the duplicates within their capacities."""
    edges = [(0, 1, 5), (0, 1, 7), (1, 2, 4), (1, 2, 4), (2, 1, 3), (1, 3, 6), (2, 3, 9), (0, 2, 2)]
    g = from_edges(4, edges, 0, 3)
    with mf.MaxFlow(g) as F:
        assert F.solve() == O.dinic(g)[0]
        check_edge_flow(F, g, g.cap)


def test_edge_flow_grid_and_rmat(mf):
    for g, inc in ((W.c2_grid_512(), 100), (W.c3_rmat20(), 1000)):
        log(f"edge flow n={g.n} m={g.m}")
        with mf.MaxFlow(g) as F:
            F.solve()
            check_edge_flow(F, g, g.cap)
            cap = g.cap.copy()
            ids, new = W.mixed_batch(cap, W.batch_size(g.m, 0.01), inc, W.rng_for(W.SEED_BASE, 42))
            cap[ids] = new
            F.update(ids, new)
            check_edge_flow(F, g, cap)
            log(f"edge flow ok, value {F.value()}")


def test_edge_flow_needs_a_solved_handle(mf):
    g = W.c1_random_1k()
    with mf.MaxFlow(g) as F:
        with pytest.raises(mf.MfError) as ei:
            F.edge_flow()
        assert ei.value.code == mf.MF_ESTATE


# ---------------- Dynamic Push-Pull ----------------

@pytest.mark.parametrize("seed", range(60))
def test_push_pull_tiny_chains(mf, seed):
    g = tiny_random(seed, n_hi=14, m_hi=50)
    with mf.MaxFlow(g, flags=mf.MF_FLAG_PUSH_PULL) as F:
        F.solve()
        check_solved(F, g, g.cap)
        rng = np.random.default_rng(1000 + seed)
        cap = g.cap.copy()
        for _ in range(4):
            if g.m == 0:
                break
            k = int(rng.integers(1, g.m + 1))
            ids = rng.choice(g.m, k, replace=False).astype(np.int64)
            new = rng.integers(0, 12, k).astype(np.int32)
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, exact_heights=False)
            if g.n <= 16:
                assert F.value() == O.brute_force_min_cut(g, cap)[0]


@pytest.mark.parametrize("grid", [1, 2, 8, 64])
@pytest.mark.parametrize("mode", [0, 1])
def test_push_pull_c1_launch_shapes(mf, grid, mode):
    g = W.c1_random_1k()
    with mf.MaxFlow(g, grid_blocks=grid, mode=mode, flags=mf.MF_FLAG_PUSH_PULL) as F:
        F.solve()
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.0125, 4, 100, seed=W.SEED_BASE + 43):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, exact_heights=False)
        check_edge_flow(F, g, cap)


@pytest.mark.parametrize("kind", ["inc", "dec", "mixed"])
def test_push_pull_update_families(mf, kind):
    g = W.rmat(15, 16, seed=44)
    frac = {"inc": 1.0, "dec": 0.0, "mixed": 0.5}[kind]
    with mf.MaxFlow(g, flags=mf.MF_FLAG_PUSH_PULL) as F, mf.MaxFlow(g) as D:
        F.solve()
        D.solve()
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.02, 3, 1000, seed=W.SEED_BASE + 44, inc_fraction=frac, p_st=0.3):
            cap[ids] = new
            v = F.update(ids, new)
            assert v == D.update(ids, new)
            check_solved(F, g, cap, exact_heights=False)
            assert np.array_equal(F.min_cut()[0], D.min_cut()[0])


def test_push_pull_grid_and_rmat_full_size(mf):
    """The 512x512 grid at 1% batches and R-MAT scale 20 at 0.1% and 1%
    batches, checked in full against the oracle."""
    g = W.c2_grid_512()
    with mf.MaxFlow(g, flags=mf.MF_FLAG_PUSH_PULL) as F:
        F.solve()
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.01, 2, 100, seed=W.SEED_BASE + 1):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, oracle="fifo", exact_heights=False)
    g = W.c3_rmat20()
    with mf.MaxFlow(g, flags=mf.MF_FLAG_PUSH_PULL) as F:
        F.solve()
        cap = g.cap.copy()
        for frac in (0.001, 0.01):
            ids, new = W.mixed_batch(cap, W.batch_size(g.m, frac), 1000,
                                     W.rng_for(W.SEED_BASE + 2, 9, int(frac * 1e4)))
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, oracle="fifo", exact_heights=False)
            log(f"push-pull rmat20 {frac}: {F.stats()['loop_kernel_ms']:.2f} ms")


def test_push_pull_errors_leave_the_handle_unchanged(mf):
    g = W.c1_random_1k()
    with mf.MaxFlow(g, flags=mf.MF_FLAG_PUSH_PULL) as F:
        v = F.solve()
        before = F.export_state()
        with pytest.raises(mf.MfError) as ei:
            F.update(np.array([3, 3], np.int64), np.array([1, 2], np.int32))
        assert ei.value.code == mf.MF_EINVAL
        for a, b in zip(before, F.export_state()):
            assert np.array_equal(a, b)
        assert F.value() == v


# ---------------- caller-supplied device memory, debug checks ----------------

def test_torch_allocator_supplies_the_handle(mf):
    g = W.c1_random_1k()
    alloc = mf.TorchAllocator()
    with mf.MaxFlow(g, allocator=alloc, flags=mf.MF_FLAG_PUSH_PULL) as F:
        # the handle's arrays, and the arc-pair build's temporaries (returned
        # before mf_create ends), all come from the allocator
        assert alloc.calls > 20 and 20 < len(alloc.live) < alloc.calls
        F.solve()
        check_solved(F, g, g.cap)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.0125, 2, 100, seed=W.SEED_BASE + 45):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, exact_heights=False)
        check_edge_flow(F, g, cap)
    assert alloc.live == {}


@pytest.mark.parametrize("fail_after", [0, 3, 12])
def test_allocation_failure_is_reported_and_cleaned_up(mf, fail_after):
    g = W.c1_random_1k()
    alloc = mf.TorchAllocator(fail_after=fail_after)
    with pytest.raises(mf.MfError) as ei:
        mf.MaxFlow(g, allocator=alloc)
    assert ei.value.code == mf.MF_ENOMEM
    assert alloc.live == {}


@pytest.mark.parametrize("flags", [0, 2])
def test_debug_checks_pass_on_every_call(mf, flags):
    g = W.rmat(13, 16, seed=46)
    with mf.MaxFlow(g, flags=4 | flags) as F:
        F.solve()
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, 0.01, 3, 1000, seed=W.SEED_BASE + 46):
            cap[ids] = new
            assert F.update(ids, new) == O.dinic(g, cap)[0]
