"""Batched solve of independent instances (one workgroup per instance, size
classes, hipGraph replay) against the oracle and against each instance
solved alone on its own handle: values bit for bit, canonical cuts element by
element."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import log
from tests.graphs import from_edges, tiny_random

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


def mixed_instances(count, seed):
    """Grids (side 4..20), random graphs (20..620 vertices, 4 edges per
    vertex) and tiny graphs with zero capacities, self-loops, duplicates,
    antiparallel edges and no s-t path."""
    out = []
    for i in range(count):
        k = seed * 1000 + i
        if i % 3 == 0:
            out.append(W.grid_instance(4 + (i * 7) % 17, k))
        elif i % 3 == 1:
            n = 20 + (i * 37) % 600
            out.append(W.random_graph(n, 4 * n, 1, 100, k, s=0, t=n - 1))
        else:
            out.append(tiny_random(k, n_hi=12, m_hi=40))
    out.append(from_edges(2, [], 0, 1))                 # no edge at all
    out.append(from_edges(3, [(1, 0, 5), (2, 1, 4)], 0, 2))  # only edges into s
    return out


def oracle_values(gs, caps=None):
    return [O.dinic(g, g.cap if caps is None else caps[i])[0] for i, g in enumerate(gs)]


@pytest.fixture(scope="module")
def mixed():
    gs = mixed_instances(45, 11)
    return gs, oracle_values(gs)


def test_batch_matches_oracle_cut_and_alone(mf, mixed):
    gs, ref = mixed
    with mf.Batch(gs) as B:
        vals = B.solve()
        assert list(vals) == ref
        for i, g in enumerate(gs):
            v, side_o, _ = O.dinic(g, g.cap)
            side, cut = B.min_cut(i)
            assert cut == v
            assert np.array_equal(side, side_o), i
    for i, g in enumerate(gs):
        with mf.MaxFlow(g) as F:
            assert F.solve() == vals[i]


@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("kc", [0, 1, 3])
@pytest.mark.parametrize("n_classes", [1, 3])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_launch_configurations(mf, mixed, block, kc, n_classes, use_graph):
    gs, ref = mixed
    with mf.Batch(gs, n_classes=n_classes, class_max_arcs=[200, 2000, 0, 0], block=[block] * 4,
                  kernel_cycles=[kc] * 4, use_graph=use_graph) as B:
        assert list(B.solve()) == ref


def test_batch_graph_replays_with_eager_work_between(mf, mixed):
    import torch
    gs, ref = mixed
    with mf.Batch(gs) as B:
        for rep in range(4):
            assert list(B.solve()) == ref, rep
            # eager work and synchronisation between replays
            with mf.MaxFlow(gs[1]) as F:
                assert F.solve() == ref[1]
            x = torch.arange(1 << 16, device="cuda", dtype=torch.int32)
            assert int(x.sum().item()) == (1 << 16) * ((1 << 16) - 1) // 2
            torch.cuda.synchronize()


def test_batch_set_capacities_follow_oracle(mf, mixed):
    gs, ref = mixed
    rng = np.random.default_rng(5)
    caps = [g.cap.copy() for g in gs]
    with mf.Batch(gs) as B:
        B.solve()
        for rnd in range(3):
            for i in rng.choice(len(gs), 10, replace=False):
                g = gs[i]
                if g.m == 0:
                    continue
                k = int(rng.integers(1, g.m + 1))
                ids = rng.choice(g.m, k, replace=False).astype(np.int64)
                new = rng.integers(0, 150, k).astype(np.int32)
                caps[i][ids] = new
                B.set_capacities(int(i), ids, new)
            assert list(B.solve()) == oracle_values(gs, caps), rnd


def test_batch_autotune_keeps_values(mf, mixed):
    gs, ref = mixed
    with mf.Batch(gs, class_max_arcs=[200, 2000, 0, 0]) as B:
        chosen = B.autotune(repeats=1)
        assert all(b in (256, 512, 1024) for b in chosen["block"][:3])
        assert list(B.solve()) == ref
        assert B.opts()["block"] == chosen["block"]


def test_batch_errors(mf, mixed):
    gs, ref = mixed
    with mf.Batch(gs[:4]) as B:
        with pytest.raises(mf.MfError) as ei:
            B.values()
        assert ei.value.code == mf.MF_ESTATE
        with pytest.raises(mf.MfError) as ei:
            B.min_cut(0)
        assert ei.value.code == mf.MF_ESTATE
        B.solve()
        with pytest.raises(mf.MfError) as ei:
            B.min_cut(9)
        assert ei.value.code == mf.MF_EINVAL
        g = gs[1]
        with pytest.raises(mf.MfError) as ei:
            B.set_capacities(1, np.array([0, 0], np.int64), np.array([1, 2], np.int32))
        assert ei.value.code == mf.MF_EINVAL and "duplicate" in str(ei.value)
        with pytest.raises(mf.MfError) as ei:
            B.set_capacities(1, np.array([g.m], np.int64), np.array([1], np.int32))
        assert ei.value.code == mf.MF_EINVAL
        # a rejected batch changes nothing
        assert list(B.solve()) == ref[:4]
        with pytest.raises(mf.MfError) as ei:
            B.set_opts(block=[100, 256, 256, 256])
        assert ei.value.code == mf.MF_EINVAL
        assert list(B.solve()) == ref[:4]


def test_c4_batch_equals_alone_and_oracle(mf):
    """All 256 instances of the uneven batch: value and canonical cut equal
    the oracle's (O2 for every instance, O1 as well for the smallest and
    largest ones), and the batched values equal single-handle solves."""
    gs = W.c4_instances()
    log(f"C4: {len(gs)} instances, sum n {sum(g.n for g in gs)}, sum m {sum(g.m for g in gs)}")
    with mf.Batch(gs) as B:
        vals = B.solve()
        log(f"C4 batch solve {B.last_ms():.2f} ms")
        again = B.solve()
        assert np.array_equal(vals, again)
        for i, g in enumerate(gs):
            v, side_o = O.fifo_push_relabel(g, g.cap)
            assert vals[i] == v, i
            side, cut = B.min_cut(i)
            assert cut == v and np.array_equal(side, side_o), i
        log("C4: every instance equals the oracle (value and canonical cut)")
        order = np.argsort([g.m for g in gs])
        for i in sorted({int(order[0]), int(order[1]), int(order[-1]), int(order[-2])}):
            assert vals[i] == O.dinic(gs[i], gs[i].cap)[0], i
    for i, g in enumerate(gs):
        with mf.MaxFlow(g) as F:
            assert F.solve() == vals[i], i
    log("C4 alone == in batch for all instances")
