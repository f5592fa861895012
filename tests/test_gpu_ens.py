"""Parity of the device MLP ensemble (FP32) with the FP64 oracle: identical
start, gradients within 1e-4 relative, trained predictions close."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
from paper_1603_04628_amd import binding as B  # noqa: E402
from oracle import mlp  # noqa: E402


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(4, 20, n), rng.uniform(0.001, 0.05, n)])
    y = 0.004 * X[:, 0] ** 2 * X[:, 1] * (1 + 0.1 * np.cos(X[:, 0])) + rng.normal(0, 0.003, n)
    return X, y


@pytest.fixture(scope="module")
def ctx():
    return hmd.Context()


def _oracle_scaled(X, y):
    mu, sd = X.mean(0), X.std(0)
    return (X - mu) / sd, y / np.sqrt(np.mean(y ** 2))


@pytest.mark.parametrize("n,hidden", [(256, 64), (37, 64), (100, 16), (2, 64), (1001, 64), (50, 1)])
def test_initial_parameters_and_gradients(ctx, n, hidden):
    X, y = data(n, n)
    cfg = B.ens_cfg(members=3, hidden=hidden, iters=1)
    Xs, ys = _oracle_scaled(X, y)
    for k in range(3):
        th_g, g_g = B.ens_grad_init(ctx, X, y, cfg, k)
        th_o = mlp.glorot_init(hidden, k, 0)
        assert np.array_equal(th_g, th_o.astype(np.float32).astype(np.float64))
        _, g_o = mlp.loss_and_grad(th_o, Xs, ys, hidden)
        assert np.linalg.norm(g_g - g_o) <= 1e-4 * np.linalg.norm(g_o)
        # tensor by tensor (W1, b1, W2, b2, W3, b3): an error confined to a
        # small tensor cannot hide behind the global norm
        H = hidden
        o = 0
        for name, size in (("W1", 2 * H), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H), ("b3", 1)):
            a, b = g_g[o:o + size], g_o[o:o + size]
            assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-9 * np.linalg.norm(g_o), (name, k)
            o += size
        assert o == len(g_o)


def test_trained_ensemble_tracks_oracle(ctx):
    X, y = data(256, 3)
    cfg = B.ens_cfg(members=5, hidden=64, iters=1500, lr=1e-3)
    e = B.Ensemble(ctx, X, y, cfg)
    o = mlp.Ensemble(X, y, members=5, hidden=64, iters=1500, lr=1e-3)
    np.testing.assert_allclose(e.losses(), o.losses, rtol=0.05, atol=1e-6)
    Xq, yq = data(200, 4)
    mg, sg = e.predict(Xq)
    mo, so = o.predict(Xq)
    rms = np.sqrt(np.mean(y ** 2))
    assert np.abs(mg - mo).max() <= 0.01 * rms
    assert np.abs(sg - so).max() <= 0.01 * rms
    # held-out targets carry noise of 0.003 (about 13% of their RMS)
    assert np.sqrt(np.mean((mg - yq) ** 2)) < 0.2 * rms


@pytest.mark.parametrize("n", [37, 256, 1001])
def test_bootstrap_gradients_match_oracle(ctx, n):
    # each member's loss weights the points by its own resample counts: the
    # same counts on both sides (Philox stream 3), tensor by tensor
    X, y = data(n, 40 + n)
    cfg = B.ens_cfg(members=3, hidden=64, iters=1, seed=17, bootstrap=1)
    Xs, ys = _oracle_scaled(X, y)
    H = 64
    for k in range(3):
        th_g, g_g = B.ens_grad_init(ctx, X, y, cfg, k)
        th_o = mlp.glorot_init(H, k, 17)
        assert np.array_equal(th_g, th_o.astype(np.float32).astype(np.float64))
        w = mlp.bootstrap_counts(n, k, 17).astype(np.float64)
        _, g_o = mlp.loss_and_grad(th_o, Xs, ys, H, w)
        _, g_plain = mlp.loss_and_grad(th_o, Xs, ys, H)
        assert np.linalg.norm(g_o - g_plain) > 1e-2 * np.linalg.norm(g_o)  # the weights matter
        o = 0
        for name, size in (("W1", 2 * H), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H), ("b3", 1)):
            a, b = g_g[o:o + size], g_o[o:o + size]
            assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-9 * np.linalg.norm(g_o), (name, k)
            o += size


def test_bootstrap_ensemble_tracks_oracle(ctx):
    X, y = data(256, 8)
    e = B.Ensemble(ctx, X, y, B.ens_cfg(members=5, hidden=64, iters=1500, lr=1e-3, bootstrap=1))
    o = mlp.Ensemble(X, y, members=5, hidden=64, iters=1500, lr=1e-3, bootstrap=True)
    np.testing.assert_allclose(e.losses(), o.losses, rtol=0.05, atol=1e-6)
    Xq, _ = data(200, 9)
    mg, sg = e.predict(Xq)
    mo, so = o.predict(Xq)
    rms = np.sqrt(np.mean(y ** 2))
    assert np.abs(mg - mo).max() <= 0.01 * rms
    # the spread is a difference of nearly equal member outputs, each of
    # which drifts from its FP64 twin over 1500 FP32 Adam steps (the
    # arithmetic of the weighted loss is pinned exactly by the gradient test)
    assert np.abs(sg - so).max() <= 0.02 * rms


def test_single_member_has_zero_spread(ctx):
    X, y = data(64, 5)
    e = B.Ensemble(ctx, X, y, B.ens_cfg(members=1, hidden=8, iters=10))
    _, s = e.predict(X[:5])
    assert np.all(s == 0.0)


def test_bad_configuration_rejected(ctx):
    X, y = data(16, 6)
    with pytest.raises(B.HmdError):
        B.Ensemble(ctx, X, y, B.ens_cfg(hidden=65))
