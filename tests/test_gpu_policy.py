"""Learned phase schedule on the GPU: the value network's forward pass and
loss gradient against the fp64 oracle, training, the phase features against
the oracle's state after the deterministic steps, and exact results under
every schedule mode."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import mlp
from tests.gpu_util import check_solved

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


def samples(N, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((N, mlp.F)).astype(np.float32)
    a = rng.integers(0, mlp.K, N).astype(np.int32)
    y = rng.normal(0, 1, N).astype(np.float32)
    return X, a, y


@pytest.mark.parametrize("N", [1, 63, 64, 1000])
def test_forward_matches_oracle(mf, N):
    with mf.Policy(seed=11) as P:
        X, _, _ = samples(N, N)
        Q = P.forward(X)
        ref = mlp.forward(P.params().astype(np.float64), X.astype(np.float64))
        assert np.allclose(Q, ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("N", [1, 64, 1000, 4097])
def test_gradient_matches_oracle(mf, N):
    """fp32 tile sums against the fp64 chain rule: relative error ~1e-4 of the
    largest gradient entry."""
    with mf.Policy(seed=N) as P:
        X, a, y = samples(N, 100 + N)
        loss, g = P.gradient(X, a, y)
        L, ref = mlp.loss_and_grad(P.params().astype(np.float64), X, a, y)
        assert loss == pytest.approx(L, rel=1e-4)
        scale = np.abs(ref).max()
        assert np.abs(g - ref).max() <= 1e-4 * scale


def test_adam_steps_match_oracle(mf):
    X, a, y = samples(500, 7)
    with mf.Policy(seed=3) as P:
        theta = P.params().astype(np.float64)
        P.train(X, a, y, steps=3, lr=1e-3)
        got = P.params()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, 4):
        _, g = mlp.loss_and_grad(theta, X, a, y)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 1e-3)
    # Adam moves each parameter by at most ~lr per step; entries whose
    # gradient is near zero may differ in sign between fp32 and fp64
    assert np.abs(got - theta).max() <= 3e-3
    assert np.mean(np.abs(got - theta) <= 1e-5) > 0.9


def test_training_fits_a_learnable_target(mf):
    rng = np.random.default_rng(1)
    X = rng.random((3000, mlp.F)).astype(np.float32)
    a = rng.integers(0, mlp.K, 3000).astype(np.int32)
    w = rng.normal(0, 1, (mlp.K, mlp.F))
    y = np.einsum("nf,nf->n", X, w[a]).astype(np.float32)
    with mf.Policy(seed=5) as P:
        l0, _ = P.gradient(X, a, y)
        l1 = P.train(X, a, y, steps=600, lr=3e-3)
        assert l1 < 0.05 * l0
        assert l1 == pytest.approx(mlp.loss(P.params().astype(np.float64), X, a, y), rel=1e-3)


def _features_now(P, batch_fraction):
    """Phase-0 features of the oracle state P (after init, or after a repair)."""
    pg = P.pg
    h = O.bfs_heights(pg, P.cf, P.e)
    levels = int(h[h < pg.n].max()) + 1
    return mlp.phase_features(pg.n, P.e, h, pg.s, pg.t, levels, 0, 0, 0, batch_fraction)


@pytest.mark.parametrize("grid", [1, 8])
def test_phase0_features_match_oracle(mf, grid):
    g = W.c1_random_1k()
    # the oracle models the repair of Alg. 5 alone: no local stage
    with mf.MaxFlow(g, grid_blocks=grid, flags=mf.MF_FLAG_GLOBAL_ONLY) as F:
        F.set_policy(None, mf.MF_POLICY_EXPLORE, explore=0.0)
        F.solve()
        tr = F.policy_trace()
        P = O.PaperSeq(g)
        P.init()
        assert tr.shape[0] >= 1
        assert np.allclose(tr[0, :16], _features_now(P, 1.0), rtol=1e-6, atol=0)
        assert tr[0, 16] == 0 and tr[0, 17] > 0
        # dynamic updates: the oracle repairs the GPU's own solved state; the
        # first update whose BFS finds active vertices records a phase
        cap = g.cap.copy()
        compared = 0
        for ids, new in W.batch_chain(g, 0.1, 6, 100, seed=W.SEED_BASE + 9):
            _, cf, e, _, _ = F.export_state()
            Q = O.PaperSeq(g, cap=cap)
            Q.cf[:] = cf
            Q.e[:] = e
            F.update(ids, new)
            cap[ids] = new
            tr = F.policy_trace()
            if tr.shape[0] == 0:
                continue
            Q.apply_updates(ids, new)
            assert np.allclose(tr[0, :16], _features_now(Q, ids.shape[0] / g.m), rtol=1e-6, atol=0)
            compared += 1
        assert compared >= 1


@pytest.mark.parametrize("mode,arg", [("forced", a) for a in range(8)] + [("explore", 0.5), ("learned", 0.0)])
@pytest.mark.parametrize("which", ["c1", "rmat13"])
def test_every_schedule_is_exact(mf, mode, arg, which):
    if which == "c1":
        g, grid, frac, inc = W.c1_random_1k(), 0, 0.0125, 100
    else:
        g, grid, frac, inc = W.rmat(13, 8, 77), 8, 0.01, 1000
    with mf.Policy(seed=9) as P, mf.MaxFlow(g, grid_blocks=grid) as F:
        if mode == "forced":
            F.set_policy(None, mf.MF_POLICY_FORCED, action=arg)
        elif mode == "explore":
            F.set_policy(None, mf.MF_POLICY_EXPLORE, explore=arg, seed=5)
        else:
            F.set_policy(P, mf.MF_POLICY_LEARNED, margin=arg)
        F.solve()
        check_solved(F, g, g.cap, full=False)
        cap = g.cap.copy()
        for ids, new in W.batch_chain(g, frac, 4, inc, seed=W.SEED_BASE + 11):
            cap[ids] = new
            F.update(ids, new)
            check_solved(F, g, cap, full=False)
            tr = F.policy_trace()
            if mode == "forced":
                assert np.all(tr[:, 16] == arg)
            assert np.all((tr[:, 16] >= 0) & (tr[:, 16] < 8))


def test_import_state_replays_an_update(mf):
    g = W.c1_random_1k()
    (ids, new), (ids2, new2) = list(W.batch_chain(g, 0.0125, 2, 100, seed=W.SEED_BASE + 21))
    with mf.MaxFlow(g) as F:
        v0 = F.solve()
        cap, cf, e, _, ecap = F.export_state()
        v1 = F.update(ids, new)
        F.import_state(cap, cf, e, ecap)
        assert F.resume() == v0
        F.import_state(cap, cf, e, ecap)
        assert F.update(ids, new) == v1 == O.dinic(g, W.apply_batch(g.cap, ids, new))[0]
        bad = cf.copy()
        bad[0] += 1
        with pytest.raises(mf.MfError) as ei:
            F.import_state(cap, bad, e, ecap)
        assert ei.value.code == mf.MF_EINVAL and "sum" in str(ei.value)
        # arc capacities must be the sums of their edges' capacities
        a = int(np.flatnonzero((cap > 0) & (cf > 0))[0])
        badcap, badcf = cap.copy(), cf.copy()
        badcap[a] -= 1
        badcf[a] -= 1  # pair sums still hold
        with pytest.raises(mf.MfError) as ei:
            F.import_state(badcap, badcf, e, ecap)
        assert ei.value.code == mf.MF_EINVAL and "edge capacities" in str(ei.value)
        badecap = ecap.copy()
        badecap[0] += 1
        with pytest.raises(mf.MfError) as ei:
            F.import_state(cap, cf, e, badecap)
        assert ei.value.code == mf.MF_EINVAL and "edge capacities" in str(ei.value)
        # excesses must equal the residual change of their vertex
        bade = e.copy()
        bade[5] += 1
        bade[6] -= 1
        with pytest.raises(mf.MfError) as ei:
            F.import_state(cap, cf, bade, ecap)
        assert ei.value.code == mf.MF_EINVAL and "excesses" in str(ei.value)
        # the rejected imports changed nothing
        F.import_state(cap, cf, e, ecap)
        assert F.update(ids, new) == v1


def test_set_policy_errors_and_fixed_mode(mf):
    g = W.c1_random_1k()
    with mf.MaxFlow(g) as F:
        for kw in (dict(mode=9), dict(mode=1), dict(mode=3, action=8), dict(mode=2, explore=1.5)):
            with pytest.raises(mf.MfError) as ei:
                F.set_policy(None, **kw)
            assert ei.value.code == mf.MF_EINVAL
        F.set_policy(None, mf.MF_POLICY_FORCED, action=3)
        F.solve()
        assert F.policy_trace().shape[0] >= 1
        F.set_policy(None, mf.MF_POLICY_FIXED)
        F.solve()
        assert F.policy_trace().shape[0] == 0
