"""Pins of the value network's oracle (oracle/mlp.py) against mathematics
that does not come from the oracle itself: central finite differences of the
loss, the closed form of linear least squares, and Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def _problem(seed, N=40):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, mlp.n_params())
    X = rng.random((N, mlp.F))
    a = rng.integers(0, mlp.K, N)
    y = rng.normal(0, 1, N)
    return theta, X, a, y


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_central_differences(seed):
    theta, X, a, y = _problem(seed)
    L, g = mlp.loss_and_grad(theta, X, a, y)
    assert L == pytest.approx(mlp.loss(theta, X, a, y), rel=1e-12)
    rng = np.random.default_rng(100 + seed)
    # every bias, and a random sample of weights from each layer
    sizes = [mlp.H * mlp.F, mlp.H, mlp.H * mlp.H, mlp.H, mlp.K * mlp.H, mlp.K]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    idx = []
    for j in range(6):
        k = sizes[j] if sizes[j] <= 32 else 24
        idx += list(offs[j] + rng.choice(sizes[j], k, replace=False))
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss(tp, X, a, y) - mlp.loss(tm, X, a, y)) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_gradient_is_linear_least_squares_when_hidden_layers_pass_through():
    """W1 = [I; 0], W2 = I, zero biases and positive inputs make h2 = [x; 0]
    and q = W3[:, :F] x + b3: the loss is then a least-squares fit whose
    gradient is (2/N) sum over the samples of action k of (q - y) x."""
    rng = np.random.default_rng(7)
    N, F, H, K = 50, mlp.F, mlp.H, mlp.K
    W1 = np.zeros((H, F)); W1[:F, :F] = np.eye(F)
    W2 = np.eye(H)
    W3 = rng.normal(0, 1, (K, H))
    b3 = rng.normal(0, 1, K)
    theta = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), b3])
    X = rng.random((N, F)) + 0.1
    a = rng.integers(0, K, N)
    y = rng.normal(0, 1, N)
    L, g = mlp.loss_and_grad(theta, X, a, y)
    pred = np.einsum("nf,nf->n", X, W3[a, :F]) + b3[a]
    assert L == pytest.approx(np.mean((pred - y) ** 2), rel=1e-12)
    gW3 = np.zeros((K, H))
    gb3 = np.zeros(K)
    for i in range(N):
        gW3[a[i], :F] += 2 * (pred[i] - y[i]) * X[i] / N
        gb3[a[i]] += 2 * (pred[i] - y[i]) / N
    o = H * F + H + H * H + H
    assert np.allclose(g[o:o + K * H].reshape(K, H), gW3, rtol=1e-12, atol=1e-14)
    assert np.allclose(g[o + K * H:], gb3, rtol=1e-12, atol=1e-14)


def test_untaken_actions_get_no_output_gradient():
    theta, X, a, y = _problem(3)
    a[:] = 2
    _, g = mlp.loss_and_grad(theta, X, a, y)
    _, _, _, _, gW3, gb3 = mlp.unpack(g)
    assert np.all(gW3[np.arange(mlp.K) != 2] == 0) and np.all(gb3[np.arange(mlp.K) != 2] == 0)


def test_adam_first_step_moves_each_parameter_by_lr():
    """With bias correction, Adam's first step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


def test_features_of_a_known_state():
    n, s, t = 6, 0, 5
    e = np.array([-9, 3, 17, 0, 70000, 4])   # vertex 4 active, vertex 2 active, 1 unreached
    h = np.array([6, 6, 2, 1, 3, 0])
    f = mlp.phase_features(n, e, h, s, t, levels=3, prev_pushes=7, prev_relabels=0, phase=1,
                           batch_fraction=0.25)
    # actives: 2 (e=17: floor log2 = 4 -> bin 1) and 4 (e=70000: 16 -> bin 4)
    assert f[0] == pytest.approx(np.log2(3) / 24)
    assert f[1] == pytest.approx(np.log2(1 + 70017) / 40, rel=1e-6)
    assert list(f[2:10]) == [0, 0.5, 0, 0, 0.5, 0, 0, 0]
    assert f[10] == pytest.approx(2 / 12)
    assert f[11] == pytest.approx(4 / 6)
    assert f[12] == pytest.approx(3 / 32) and f[13] == 0
    assert f[14] == pytest.approx(1 / 8) and f[15] == pytest.approx(0.25)
