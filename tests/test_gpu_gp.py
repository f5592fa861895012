"""Parity of the device GP (FP64) with the oracle GP through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
from paper_1603_04628_amd import binding as B  # noqa: E402
from oracle.gp import GP as OGP, Hyper  # noqa: E402

RANGES = (16.0, 0.049)


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(4, 20, n), rng.uniform(0.001, 0.05, n)])
    y = 0.002 * X[:, 0] ** 3 * X[:, 1] * (1 + 0.2 * np.sin(X[:, 0])) + rng.normal(0, 0.01, n)
    se = rng.uniform(0.005, 0.02, n)
    return X, y, se


@pytest.fixture(scope="module")
def ctx():
    return hmd.Context()


@pytest.mark.parametrize("n", [1, 2, 7, 64, 65, 256, 333])
def test_fit_predict_matches_oracle(ctx, n):
    X, y, se = data(n, n)
    g = B.GP(ctx, X, y, se, B.gp_hyper(ranges=RANGES))
    o = OGP(X, y, se, Hyper(ranges=RANGES))
    sc, sq, sn = g.scales()
    np.testing.assert_allclose(sc, o.scale, rtol=1e-13)
    assert sq == pytest.approx(o.s_q, rel=1e-14) and sn == pytest.approx(o.sigma_n, rel=1e-13)
    Xs, _, _ = data(200, 1000 + n)
    Xs = np.vstack([Xs, X[:3], [[40.0, 0.2]]])
    mg, vg = g.predict(Xs)
    mo, vo = o.predict(Xs)
    scale = max(np.abs(mo).max(), 1e-30)
    assert np.abs(mg - mo).max() <= 1e-9 * scale + 1e-12
    assert np.abs(vg - vo).max() <= 1e-9 * o.s_q ** 2
    assert g.log_marginal() == pytest.approx(o.log_marginal(), rel=1e-9, abs=1e-9)


def test_append_matches_oracle_refit(ctx):
    X, y, se = data(40, 7)
    g = B.GP(ctx, X[:30], y[:30], se[:30], B.gp_hyper(ranges=RANGES))
    o = OGP(X[:30], y[:30], se[:30], Hyper(ranges=RANGES))
    for k in range(30, 40):
        g.append(X[k], y[k], se[k])
        o.append(X[k], y[k], se[k])
    assert len(g) == 40
    Xs, _, _ = data(50, 99)
    np.testing.assert_allclose(g.predict(Xs)[0], o.predict(Xs)[0], rtol=1e-9, atol=1e-12)


def test_rank_one_append_equals_full_factorisation(ctx):
    X, y, _ = data(70, 8)
    hp = B.gp_hyper(sigma_n=0.05, scale_mode=1, ranges=RANGES, out_scale=0)
    g = B.GP(ctx, X[:60], y[:60], None, hp)
    for k in range(60, 70):
        g.append(X[k], y[k], 0.0)
    full = B.GP(ctx, X, y, None, hp)
    Xs, _, _ = data(30, 5)
    a, b = g.predict(Xs), full.predict(Xs)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10, atol=1e-13)
    o = OGP(X, y, None, Hyper(sigma_n=0.05, scale_mode=1, ranges=RANGES, out_scale=0))
    np.testing.assert_allclose(a[0], o.predict(Xs)[0], rtol=1e-9, atol=1e-12)


def test_empty_database_returns_prior(ctx):
    g = B.GP(ctx, np.zeros((0, 2)), np.zeros(0), None, B.gp_hyper(ranges=RANGES))
    m, v = g.predict([[5.0, 0.01], [10.0, 0.02]])
    assert np.all(m == 0.0) and np.all(v == 1.0)
    g.append([5.0, 0.01], 0.3, 0.01)
    m, v = g.predict([[5.0, 0.01]])
    assert v[0] < 1.0


def test_duplicate_points_without_noise_are_not_spd(ctx):
    X = np.array([[5.0, 0.01], [5.0, 0.01]])
    with pytest.raises(B.HmdError) as e:
        B.GP(ctx, X, [0.1, 0.1], None, B.gp_hyper(sigma_n=0.0, ranges=RANGES))
    assert e.value.code == B.HMD_ENOTSPD


def test_database_size_limit(ctx):
    X = np.column_stack([np.linspace(4, 20, 6145), np.full(6145, 0.01)])
    with pytest.raises(B.HmdError) as e:
        B.GP(ctx, X, np.zeros(6145), None, B.gp_hyper(ranges=RANGES))
    assert e.value.code == B.HMD_EINVAL


def test_long_rank_one_append_chain(ctx):
    """L^-1 extended row by row over many appends stays equal to a fresh inverse."""
    X, y, _ = data(300, 11)
    hp = B.gp_hyper(sigma_n=0.05, scale_mode=1, ranges=RANGES, out_scale=0)
    g = B.GP(ctx, X[:2], y[:2], None, hp)
    for k in range(2, 300):
        g.append(X[k], y[k], 0.0)
    full = B.GP(ctx, X, y, None, hp)
    Xs, _, _ = data(64, 12)
    a, b = g.predict(Xs), full.predict(Xs)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-9, atol=1e-12)


def test_large_database_matches_oracle(ctx):
    """2050 points (a ragged tail on every 256-thread loop and 32 x 32 tile),
    fixed scales and noise so the covariance stays well conditioned."""
    X, y, _ = data(2050, 21)
    hp = B.gp_hyper(sigma_n=0.05, scale_mode=1, ranges=RANGES, out_scale=0)
    g = B.GP(ctx, X, y, None, hp)
    o = OGP(X, y, None, Hyper(sigma_n=0.05, scale_mode=1, ranges=RANGES, out_scale=0))
    Xs, _, _ = data(300, 22)
    mg, vg = g.predict(Xs)
    mo, vo = o.predict(Xs)
    assert np.abs(mg - mo).max() <= 1e-9 * np.abs(mo).max() + 1e-12
    assert np.abs(vg - vo).max() <= 1e-9
    assert g.log_marginal() == pytest.approx(o.log_marginal(), rel=1e-9, abs=1e-9)


def test_database_at_the_size_limit_matches_oracle(ctx):
    """6144 points, the largest database the device GP takes; noise 0.2 keeps
    cond(C) below 1 + n / 0.2^2 ~ 1.5e5."""
    X, y, _ = data(6144, 23)
    hp = B.gp_hyper(sigma_n=0.2, scale_mode=1, ranges=RANGES, out_scale=0)
    g = B.GP(ctx, X, y, None, hp)
    assert len(g) == 6144
    o = OGP(X, y, None, Hyper(sigma_n=0.2, scale_mode=1, ranges=RANGES, out_scale=0))
    Xs, _, _ = data(64, 24)
    mg, vg = g.predict(Xs)
    mo, vo = o.predict(Xs)
    assert np.abs(mg - mo).max() <= 1e-9 * np.abs(mo).max() + 1e-12
    assert np.abs(vg - vo).max() <= 1e-9


def test_many_queries_match_oracle(ctx):
    """4097 queries (one workgroup each, a ragged count) on a 256-point database."""
    X, y, se = data(256, 31)
    g = B.GP(ctx, X, y, se, B.gp_hyper(ranges=RANGES))
    o = OGP(X, y, se, Hyper(ranges=RANGES))
    Xs, _, _ = data(4097, 32)
    mg, vg = g.predict(Xs)
    mo, vo = o.predict(Xs)
    assert np.abs(mg - mo).max() <= 1e-9 * np.abs(mo).max() + 1e-12
    assert np.abs(vg - vo).max() <= 1e-9 * o.s_q ** 2


# ---------------------------------------------------------------- NEXT-4 options
@pytest.mark.parametrize("n", [1, 40, 300])
def test_heteroscedastic_noise_matches_oracle(ctx, n):
    X, y, se = data(n, 500 + n)
    se = se * np.linspace(0.2, 5.0, n)  # very uneven per-point errors
    g = B.GP(ctx, X, y, se, B.gp_hyper(ranges=RANGES, noise_mode=1))
    o = OGP(X, y, se, Hyper(ranges=RANGES, noise_mode=1))
    Xs, _, _ = data(150, 900 + n)
    mg, vg = g.predict(Xs)
    mo, vo = o.predict(Xs)
    assert np.abs(mg - mo).max() <= 1e-9 * np.abs(mo).max() + 1e-12
    assert np.abs(vg - vo).max() <= 1e-9 * vo.max()
    assert g.log_marginal() == pytest.approx(o.log_marginal(), rel=1e-10)
    # appending keeps matching (a refit: the normalisation moves)
    g.append(Xs[0], 0.01, 0.5)
    o.append(Xs[0], 0.01, 0.5)
    assert np.abs(g.predict(Xs)[0] - o.predict(Xs)[0]).max() <= 1e-9 * np.abs(mo).max() + 1e-12


def test_heteroscedastic_rank_one_append_equals_refit(ctx):
    X, y, se = data(50, 77)
    hp = dict(ranges=RANGES, scale_mode=1, out_scale=0, noise_mode=1)
    g = B.GP(ctx, X[:30], y[:30], se[:30], B.gp_hyper(**hp))
    for k in range(30, 50):
        g.append(X[k], y[k], se[k])
    full = B.GP(ctx, X, y, se, B.gp_hyper(**hp))
    Xs, _, _ = data(60, 78)
    assert np.allclose(g.predict(Xs)[0], full.predict(Xs)[0], rtol=1e-9, atol=1e-12)
    assert np.allclose(g.predict(Xs)[1], full.predict(Xs)[1], rtol=1e-8, atol=1e-14)


def test_periodic_kernel_matches_oracle(ctx):
    # App. B: a noisy sinusoidal time series smoothed with the periodic kernel
    T = 10.8
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0.0, 25.0, 120))[:, None]
    y = np.sin(2 * np.pi * t[:, 0] / T) + 0.2 * rng.standard_normal(120)
    hp = dict(sigma_n=0.2, out_scale=0, kernel=1, period=T, ranges=(1.0,))
    g = B.GP(ctx, t, y, None, B.gp_hyper(**hp))
    o = OGP(t, y, None, Hyper(**hp))
    q = np.linspace(0.0, 40.0, 81)[:, None]
    mg, vg = g.predict(q)
    mo, vo = o.predict(q)
    assert np.abs(mg - mo).max() <= 1e-9
    assert np.abs(vg - vo).max() <= 1e-9
    assert g.log_marginal() == pytest.approx(o.log_marginal(), rel=1e-10)
    with pytest.raises(hmd.HmdError):  # the periodic kernel takes one input
        B.GP(ctx, np.column_stack([t, t]), y, None, B.gp_hyper(**hp))


@pytest.mark.parametrize("which,kernel", [(("sigma_f", "ell"), 0), (("ell", "sigma_n"), 1)])
def test_optimised_hyperparameters_match_oracle(ctx, which, kernel):
    rng = np.random.default_rng(11)
    if kernel == 0:
        X, y, se = data(80, 12)
        hp = dict(ranges=RANGES)
        sen = se
    else:
        T = 10.8
        X = np.sort(rng.uniform(0.0, 25.0, 60))[:, None]
        y = np.sin(2 * np.pi * X[:, 0] / T) + 0.15 * rng.standard_normal(60)
        hp = dict(sigma_n=0.3, out_scale=0, kernel=1, period=T, ranges=(1.0,))
        sen = None
    g = B.GP(ctx, X, y, sen, B.gp_hyper(**hp))
    o = OGP(X, y, sen, Hyper(**hp))
    lg = g.optimize(which)
    lo = o.optimize(which)
    assert lg == pytest.approx(lo, rel=1e-8, abs=1e-8)
    hg = g.hyper()
    for k in which:
        ref = o.h.sigma_n if k == "sigma_n" else getattr(o.h, k)
        assert hg[k] == pytest.approx(ref, rel=2e-3), k
    assert g.log_marginal() == pytest.approx(lg, rel=1e-12)
    Xs = X[:10] + 0.01
    assert np.abs(g.predict(Xs)[0] - o.predict(Xs)[0]).max() <= 1e-4 * np.abs(y).max()


def test_database_copy_round_trips(ctx):
    # gp_inputs + gp_outputs return the database as given (fit, then
    # appends), and a GP fitted to that copy answers exactly as the original
    X, y, se = data(40, 11)
    hp = B.gp_hyper(ranges=RANGES, sigma_n=0.01, scale_mode=1, out_scale=0)
    g = B.GP(ctx, X[:30], y[:30], se[:30], hp)
    for k in range(30, 40):
        g.append(X[k], y[k], se[k])
    Xc, yc, sc = g.data()
    assert np.array_equal(Xc, X) and np.array_equal(yc, y) and np.array_equal(sc, se)
    c = B.GP(ctx, Xc, yc, sc, hp)
    Xs, _, _ = data(50, 12)
    m0, v0 = g.predict(Xs)
    m1, v1 = c.predict(Xs)
    np.testing.assert_allclose(m1, m0, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(v1, v0, rtol=1e-6, atol=1e-14)
    e = B.GP(ctx, np.zeros((0, 2)), np.zeros(0), np.zeros(0), hp)
    assert len(e) == 0 and all(len(a) == 0 for a in e.data())


def test_time_series_smoother_matches_oracle(ctx):
    # the App. B smoother as the study runner applies it to the all-MD
    # march's flux series (two forcing periods, outputs scaled by their RMS,
    # sigma_f, ell and sigma_n all by the evidence), on a 100-step series:
    # the maximum and the smoothed series agree with the oracle's
    rng = np.random.default_rng(21)
    t = np.arange(100, dtype=np.float64)[:, None]
    y = 0.04 * np.sin(2 * np.pi * t[:, 0] / 50.0) + 0.004 * rng.standard_normal(100)
    hp = dict(kernel=1, period=50.0, out_scale=1, sigma_n=0.1 * float(np.std(y)), ranges=(100.0,))
    g = B.GP(ctx, t, y, None, B.gp_hyper(**hp))
    o = OGP(t, y, None, Hyper(**hp))
    which = ("sigma_f", "ell", "sigma_n")
    lg = g.optimize(which)
    lo = o.optimize(which)
    # three hyperparameters over a flat, correlated maximum: the device's
    # cyclic golden-section searches and the oracle's Nelder-Mead stop
    # within 1e-6 of it (relative), and the smoothed series within 1e-3 of
    # its peak, ten times below what the smoothing leaves of the noise
    assert lg == pytest.approx(lo, rel=1e-6)
    Qg, _ = g.predict(t)
    Qo, _ = o.predict(t)
    assert np.abs(Qg - Qo).max() <= 1e-3 * np.abs(Qo).max()
    # the smoothing removes most of the noise: the residual to the noiseless
    # signal is well below the noise level
    clean = 0.04 * np.sin(2 * np.pi * t[:, 0] / 50.0)
    assert np.sqrt(np.mean((Qg - clean) ** 2)) < 0.5 * 0.004
