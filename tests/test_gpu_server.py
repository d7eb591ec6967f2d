"""Serving runtime on the GPU: every committed (value, version) equals the
oracle's maximum flow after the graph's first `version` requests, whether the
graph is served alone or among other tenants, with or without group commit."""
import threading
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


def tenant(kind, seed):
    if kind == "random":
        return W.random_graph(800, 6400, 1, 100, seed)
    if kind == "grid":
        return W.grid_instance(40, seed)
    return W.rmat(12, 8, seed)


@pytest.fixture(scope="module")
def tenants():
    """Three graphs, 25 requests each, and the oracle value after every
    prefix of each graph's requests."""
    out = []
    for j, kind in enumerate(("random", "grid", "rmat")):
        g = tenant(kind, 300 + j)
        reqs = list(W.request_stream(g, 25, 400 + j, k_lo=1, k_hi=min(400, g.m)))
        cap = g.cap.copy()
        prefix = [O.dinic(g, cap)[0]]
        for ids, new in reqs:
            cap[ids] = new
            prefix.append(O.dinic(g, cap)[0])
        out.append((g, reqs, prefix))
    return out


def check_results(results, prefix, nreq):
    seqs = sorted(r["seq"] for r in results)
    assert seqs == list(range(1, nreq + 1))
    for r in results:
        assert r["status"] == 0, r
        assert r["seq"] <= r["version"] <= nreq
        assert r["value"] == prefix[r["version"]], r
        assert r["submit_ms"] <= r["start_ms"] <= r["done_ms"]


def serve(mf, tenants, which, workers, group, jitter):
    """Submit each chosen tenant's requests from its own thread (optionally
    with random pauses), then wait for all; returns {tenant: results}."""
    res = {}
    with mf.Server(workers=workers, max_group_requests=group) as S:
        gids = {}
        for j in which:
            g, reqs, prefix = tenants[j]
            gid, v0 = S.add_graph(g)
            assert v0 == prefix[0]
            gids[j] = gid

        def run(j):
            rng = np.random.default_rng(j)
            rids = []
            for ids, new in tenants[j][1]:
                rids.append(S.submit(gids[j], ids, new))
                if jitter:
                    time.sleep(float(rng.exponential(0.002)))
            res[j] = [S.wait(r) for r in rids]

        th = [threading.Thread(target=run, args=(j,)) for j in which]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for j in which:
            assert S.graph_info(gids[j]) == (len(tenants[j][1]), tenants[j][2][-1])
        mem = S.memory()
        assert mem["reserved"] > 0 and mem["commits"] >= 1
    return res


def test_alone_with_group_commit(mf, tenants):
    res = serve(mf, tenants, [0], workers=1, group=64, jitter=False)
    check_results(res[0], tenants[0][2], 25)
    # all requests were queued at once: at least one commit merged several
    assert max(r["group_size"] for r in res[0]) > 1


def test_alone_without_group_commit(mf, tenants):
    res = serve(mf, tenants, [0], workers=1, group=1, jitter=False)
    check_results(res[0], tenants[0][2], 25)
    assert all(r["version"] == r["seq"] and r["group_size"] == 1 for r in res[0])


def test_mix_equals_alone(mf, tenants):
    alone = {j: serve(mf, tenants, [j], workers=1, group=64, jitter=True)[j] for j in range(3)}
    mix = serve(mf, tenants, [0, 1, 2], workers=4, group=64, jitter=True)
    for j in range(3):
        check_results(mix[j], tenants[j][2], 25)
        by_version = {r["version"]: r["value"] for r in alone[j]}
        for r in mix[j]:
            if r["version"] in by_version:
                assert r["value"] == by_version[r["version"]]


def test_admission_by_memory_budget(mf, tenants):
    small, big = tenants[0][0], tenants[2][0]
    need_small = mf.mf_estimate_device_bytes(small.n, small.m) + 12 * small.m
    with mf.Server(workers=2, memory_budget=need_small + 1000) as S:
        gid, _ = S.add_graph(small)
        before = S.memory()["reserved"]
        with pytest.raises(mf.MfError) as ei:
            S.add_graph(big)
        assert ei.value.code == mf.MF_ENOMEM and "admission" in str(ei.value)
        assert S.memory()["reserved"] == before
        S.remove_graph(gid)
        assert S.memory()["reserved"] == 0
        with pytest.raises(mf.MfError):
            S.submit(gid, np.array([0], np.int64), np.array([1], np.int32))
        gid2, v = S.add_graph(small)
        assert v == tenants[0][2][0]


def test_submit_errors(mf, tenants):
    g, reqs, prefix = tenants[0]
    with mf.Server(workers=1) as S:
        gid, _ = S.add_graph(g)
        for ids, caps, what in (([0, 0], [1, 2], "duplicate"), ([g.m], [1], "out of range"),
                                ([1], [1 << 30], "capacity outside")):
            with pytest.raises(mf.MfError) as ei:
                S.submit(gid, np.array(ids, np.int64), np.array(caps, np.int32))
            assert ei.value.code == mf.MF_EINVAL and what in str(ei.value)
        with pytest.raises(mf.MfError):
            S.submit(gid + 7, np.array([0], np.int64), np.array([1], np.int32))
        with pytest.raises(mf.MfError):
            S.poll(12345)
        rid = S.submit(gid, *reqs[0])
        r = S.wait(rid)
        assert r["version"] == 1 and r["value"] == prefix[1]
        assert S.poll(rid)["value"] == prefix[1]
        # a released result is gone; releasing it again or polling it is an error
        assert S.release(rid)
        for call in (S.poll, S.release):
            with pytest.raises(mf.MfError) as ei:
                call(rid)
            assert ei.value.code == mf.MF_EINVAL


def test_mix_of_multi_workgroup_tenants(mf):
    """Two tenants whose solve kernels are cooperative grids of several
    workgroups (above the one-workgroup size), served alone and together:
    every commit equals the oracle's prefix value, and the grids in flight
    never exceed the device's workgroup slots."""
    graphs = [W.rmat(15, 8, seed=501), W.grid_instance(160, seed=502)]
    streams, prefixes = [], []
    for j, g in enumerate(graphs):
        with mf.MaxFlow(g) as F:
            F.solve()
            assert F.stats()["grid_blocks"] > 1
        reqs = list(W.request_stream(g, 12, 600 + j, k_lo=10, k_hi=5000))
        cap = g.cap.copy()
        prefix = [O.dinic(g, cap)[0]]
        for ids, new in reqs:
            cap[ids] = new
            prefix.append(O.dinic(g, cap)[0])
        streams.append(reqs)
        prefixes.append(prefix)

    def run(which):
        res = {}
        with mf.Server(workers=4) as S:
            gids = {j: S.add_graph(graphs[j])[0] for j in which}
            assert S.load()["slots"] >= 16

            def go(j):
                rids = [S.submit(gids[j], ids, new) for ids, new in streams[j]]
                res[j] = [S.wait(r) for r in rids]

            th = [threading.Thread(target=go, args=(j,)) for j in which]
            for t in th:
                t.start()
            for t in th:
                t.join()
            load = S.load()
            assert load["slots_used"] == 0 and load["pending_bytes"] == 0
        return res

    alone = {j: run([j])[j] for j in range(2)}
    mix = run([0, 1])
    for j in range(2):
        check_results(alone[j], prefixes[j], len(streams[j]))
        check_results(mix[j], prefixes[j], len(streams[j]))


def test_request_admission(mf, tenants):
    g, reqs, prefix = tenants[0]
    with mf.Server(workers=1, max_pending_bytes=12 * 50, max_group_edges=200) as S:
        gid, _ = S.add_graph(g)
        ids = np.arange(100, dtype=np.int64)
        caps = g.cap[:100].copy()
        # a request whose own bytes exceed the queue's limit is turned away, untouched
        with pytest.raises(mf.MfError) as ei:
            S.submit(gid, ids, caps)
        assert ei.value.code == mf.MF_EBUSY and "admission" in str(ei.value)
        # more edges than one commit stages
        with pytest.raises(mf.MfError) as ei:
            S.submit(gid, np.arange(300, dtype=np.int64), g.cap[:300].copy())
        assert ei.value.code == mf.MF_EINVAL and "max_group_edges" in str(ei.value)
        r = S.wait(S.submit(gid, ids[:40], caps[:40]))
        assert r["status"] == 0 and r["value"] == prefix[0]
        assert S.load()["pending_bytes"] == 0
