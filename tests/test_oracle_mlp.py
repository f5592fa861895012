"""Pins for the MLP-ensemble oracle: finite-difference gradients, the Adam
update formula, the Glorot-uniform start, and that training fits.  CPU only."""
import numpy as np
import pytest

from oracle import md as omd
from oracle import mlp


def _data(n=64, seed=0):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(4, 20, n), rng.uniform(0.001, 0.05, n)])
    y = 0.003 * X[:, 0] ** 2 * X[:, 1] * 10
    return X, y


def test_backward_matches_central_differences():
    H = 8
    rng = np.random.default_rng(1)
    theta = rng.normal(0, 0.5, mlp.n_params(H))
    Xs = rng.normal(size=(10, 2))
    ys = rng.normal(size=10)
    _, g = mlp.loss_and_grad(theta, Xs, ys, H)
    fd = np.zeros_like(theta)
    h = 1e-6
    for p in range(len(theta)):
        e = np.zeros_like(theta)
        e[p] = h
        fd[p] = (mlp.loss_and_grad(theta + e, Xs, ys, H)[0] - mlp.loss_and_grad(theta - e, Xs, ys, H)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_first_adam_step_is_lr_times_sign():
    # with m = v = 0 the bias-corrected first step is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_glorot_uniform_start():
    H = 64
    th = mlp.glorot_init(H, 0, 0)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, H)
    for W, lim in ((W1, np.sqrt(6 / 66)), (W2, np.sqrt(6 / 128)), (W3, np.sqrt(6 / 65))):
        assert np.abs(W).max() < lim
        assert np.var(W) == pytest.approx(lim ** 2 / 3, rel=0.2 if W.size > 100 else 0.6)
    assert not b1.any() and not b2.any() and not b3.any()
    assert not np.array_equal(th, mlp.glorot_init(H, 1, 0))
    assert np.array_equal(th, mlp.glorot_init(H, 0, 0))


def test_ensemble_fits_a_smooth_map():
    X, y = _data(64)
    ens = mlp.Ensemble(X, y, members=2, hidden=16, iters=1500, lr=3e-3)
    assert max(ens.losses) < 1e-3
    m, s = ens.predict(X)
    assert np.sqrt(np.mean((m - y) ** 2)) < 0.05 * np.sqrt(np.mean(y ** 2))
    assert np.all(s >= 0)


def test_forward_of_a_hand_set_network():
    # H = 2, input (0.5, -1), flat layout W1 [H x 2] (one row per hidden
    # unit), b1, W2 [H x H], b2, W3 [1 x H], b3:
    #   W1 = [[2, 1], [0, -3]], b1 = (0, -2):  z1 = (0, 1), h1 = (0, t), t = tanh 1
    #   W2 = [[1, 2], [-1, 0.5]], b2 = (0.25, 0):  h2 = (tanh(2t + 1/4), tanh(t/2))
    #   W3 = [3, -2], b3 = 0.1:  out = 3 tanh(2t + 1/4) - 2 tanh(t/2) + 0.1
    # = 2.205074484369277.  A transposed W1 or W2, or a bias in the wrong
    # slot, changes the value.
    theta = np.array([2.0, 1.0, 0.0, -3.0, 0.0, -2.0,
                      1.0, 2.0, -1.0, 0.5, 0.25, 0.0,
                      3.0, -2.0, 0.1])
    assert len(theta) == mlp.n_params(2)
    out, (h1, h2) = mlp.forward(theta, np.array([[0.5, -1.0]]), 2)
    assert out[0] == pytest.approx(2.205074484369277, abs=1e-14)
    assert h1[0, 0] == 0.0 and h1[0, 1] == pytest.approx(0.7615941559557649, abs=1e-15)
    # the ensemble applies the input standardisation and output scale around
    # the same network: inputs (mu + sd x) and outputs s_q out
    ens = mlp.Ensemble.__new__(mlp.Ensemble)
    ens.H, ens.mu, ens.sd, ens.s_q, ens.thetas = 2, np.array([1.0, 2.0]), np.array([4.0, 0.5]), 3.0, [theta]
    m = ens.member_predict(np.array([[1.0 + 4.0 * 0.5, 2.0 + 0.5 * -1.0]]))
    assert m[0, 0] == pytest.approx(3.0 * 2.205074484369277, abs=1e-13)


def test_bootstrap_weights_equal_an_explicit_resample():
    # the weighted loss is the plain MSE over the resampled set itself: the
    # drawn indices, read straight from the Philox words, give the same loss
    # and gradient when the points are repeated explicitly
    H, N, seed, member = 6, 37, 99, 3
    rng = np.random.default_rng(2)
    theta = rng.normal(0, 0.5, mlp.n_params(H))
    Xs = rng.normal(size=(N, 2))
    ys = rng.normal(size=N)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    idx = []
    for j in range((N + 3) // 4):
        r = omd.philox4x32_10([j, member, 3, 0], key)
        idx += [(int(w) * N) >> 32 for w in r]
    idx = np.array(idx[:N])
    c = mlp.bootstrap_counts(N, member, seed)
    assert c.sum() == N and np.array_equal(c, np.bincount(idx, minlength=N))
    lw, gw = mlp.loss_and_grad(theta, Xs, ys, H, c)
    lr, gr = mlp.loss_and_grad(theta, Xs[idx], ys[idx], H)
    assert lw == pytest.approx(lr, rel=1e-12)
    np.testing.assert_allclose(gw, gr, rtol=1e-10, atol=1e-14)


def test_bootstrap_draws_are_uniform_and_members_differ():
    # multinomial(N, 1/N): about 1 - 1/e of the points appear; the counts
    # follow Poisson(1) in the large-N limit; members draw independently
    N = 20000
    c0, c1 = mlp.bootstrap_counts(N, 0, 5), mlp.bootstrap_counts(N, 1, 5)
    assert (c0 > 0).mean() == pytest.approx(1.0 - np.exp(-1.0), abs=0.01)
    for k in range(4):
        p = np.exp(-1.0) / np.prod(np.arange(1, k + 1)) if k else np.exp(-1.0)
        assert (c0 == k).mean() == pytest.approx(p, abs=0.01)
    assert np.corrcoef(c0, c1)[0, 1] == pytest.approx(0.0, abs=0.03)
