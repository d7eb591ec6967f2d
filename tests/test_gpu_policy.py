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
    with mf.MaxFlow(g, grid_blocks=grid) as F:
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


# ---------------- the learned schedule against the fixed rule ----------------

_FRACTIONS = (0.001, 0.01, 0.1)


def _chain(g, count, seed):
    cur = g.cap.copy()
    for j in range(count):
        k = W.batch_size(g.m, _FRACTIONS[j % 3])
        ids, new = W.mixed_batch(cur, k, 1000, W.rng_for(seed, 1, j))
        cur[ids] = new
        yield ids, new


def _collect_paired(mf, g, count, seed):
    """Every update call of a chain is replayed from the same state (export,
    import) under each of the 8 actions held for the whole call; sample =
    (features of the call's first phase, action, log of the call's loop time
    over the time under action 0).  The chain then goes on under the fixed
    rule.  Calls whose first global relabel finds no active vertex have no
    phase and give no sample."""
    X, A, Y = [], [], []
    with mf.MaxFlow(g) as F:
        F.solve()
        for ids, new in _chain(g, count, seed):
            cap, cf, e, _, ecap = F.export_state()
            times, feats, values = [], None, set()
            for a in range(8):
                F.import_state(cap, cf, e, ecap)
                F.set_policy(None, mf.MF_POLICY_FORCED, action=a)
                values.add(F.update(ids, new))
                tr = F.policy_trace()
                if tr.shape[0] == 0:
                    break
                if feats is None:
                    feats = tr[0, :16].copy()
                assert np.array_equal(tr[0, :16], feats)  # same state, same first phase
                times.append(F.stats()["loop_kernel_ms"])
            assert len(values) == 1
            if len(times) == 8:
                for a in range(8):
                    X.append(feats)
                    A.append(a)
                    Y.append(np.log(times[a] / times[0]))
            F.import_state(cap, cf, e, ecap)
            F.set_policy(None, mf.MF_POLICY_FIXED)
            F.update(ids, new)
    return np.array(X, np.float32), np.array(A, np.int32), np.array(Y, np.float32)


def _paired_eval(mf, g, count, seed, policy, acts):
    """Every call of a held-out chain is replayed from one exported state
    under the fixed rule and under the learned schedule (the order alternates
    from call to call); both must give the same value.  Returns the loop time
    of the chain under each."""
    tf = tl = 0.0
    with mf.MaxFlow(g) as F:
        F.solve()
        for j, (ids, new) in enumerate(_chain(g, count, seed)):
            cap, cf, e, _, ecap = F.export_state()
            vals = {}
            for which in ((0, 1) if j % 2 == 0 else (1, 0)):
                F.import_state(cap, cf, e, ecap)
                if which == 0:
                    F.set_policy(None, mf.MF_POLICY_FIXED)
                else:
                    F.set_policy(policy, mf.MF_POLICY_LEARNED | mf.MF_POLICY_PER_CALL, margin=0.05)
                vals[which] = F.update(ids, new)
                ms = F.stats()["loop_kernel_ms"]
                if which == 0:
                    tf += ms
                else:
                    tl += ms
                    tr = F.policy_trace()
                    if tr.shape[0]:
                        acts.append(int(tr[0, 16]))
            assert vals[0] == vals[1]
    return tf, tl


def test_learned_schedule_beats_the_fixed_rule_on_held_out_graphs(mf):
    """Trained on R-MAT graphs (seeds 900..904) and segmentation grids of
    sides 128..224 (seeds 40..45), evaluated on held-out seeds of both
    families; update chains mix
    0.1 %, 1 % and 10 % batches.  The training signal is paired: each call is
    replayed from one state under every action, and the target is the log
    ratio of its loop time to the fixed rule's.  The best action differs by
    family and batch size (a shorter relabel budget on grids, longer phases
    on R-MAT at large batches), which one rule cannot serve.  The learned
    per-call schedule must need less loop time than the fixed rule in total,
    with every call of the held-out chains replayed from the same state under
    both (medians of three repetitions per graph) and identical values."""
    train = [W.rmat(16, 16, 900 + i) for i in range(3)] + [W.rmat(17, 16, 903 + i) for i in range(2)]
    train += [W.seg_grid(128, seed=40), W.seg_grid(160, seed=41), W.seg_grid(160, seed=42),
              W.seg_grid(192, seed=43), W.seg_grid(208, seed=44), W.seg_grid(224, seed=45)]
    data = [_collect_paired(mf, g, 18, 50 + i) for i, g in enumerate(train)]
    X = np.concatenate([d[0] for d in data])
    A = np.concatenate([d[1] for d in data])
    Y = np.concatenate([d[2] for d in data])
    assert len(np.unique(A)) == 8
    with mf.Policy(seed=1) as P:
        l0, _ = P.gradient(X, A, Y)
        l1 = P.train(X, A, Y, steps=2000, lr=3e-3)
        assert l1 < l0
        fixed_total = learned_total = 0.0
        evals = [W.rmat(17, 16, 990), W.rmat(18, 16, 991), W.seg_grid(192, seed=70), W.seg_grid(224, seed=71)]
        for gi, g in enumerate(evals):
            tf, tl, acts = [], [], []
            for rep in range(3):
                a, b = _paired_eval(mf, g, 12, 7 + gi, P, acts)
                tf.append(a)
                tl.append(b)
            fixed_total += float(np.median(tf))
            learned_total += float(np.median(tl))
            print(f"  graph {gi}: fixed {np.median(tf):.1f} ms, learned {np.median(tl):.1f} ms, "
                  f"actions {np.bincount(acts, minlength=8).tolist()}")
        gain = fixed_total / learned_total
        print(f"learned schedule: fixed {fixed_total:.1f} ms, learned {learned_total:.1f} ms, gain {gain:.3f}x")
        assert learned_total < fixed_total
