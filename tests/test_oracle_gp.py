"""Pins for the GP oracle (Sec. 2.2-2.3 of the paper) against closed forms,
limits and independent library routines.  CPU only."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle.gp import GP, Hyper, mean_separation


def fixed(sigma_n=0.1, sigma_f=1.0, ell=1.0, ranges=(4.0, 4.0)):
    # fixed normalisation and no output scaling: bare Eqs. covarianceEq-evidenceEq
    return Hyper(sigma_f=sigma_f, ell=ell, sigma_n=sigma_n, scale_mode=1, ranges=ranges, out_scale=0)


def test_single_point_closed_form():
    gp = GP([[1.0, 2.0]], [0.7], hyper=fixed(sigma_n=0.3))
    xs = np.array([[1.5, 1.0]])
    # scale = range/4 = 1 per input: d^2 = 0.25 + 1
    k = np.exp(-0.5 * 1.25)
    m, v = gp.predict(xs)
    assert m[0] == pytest.approx(k * 0.7 / (1.0 + 0.09), rel=1e-14)
    assert v[0] == pytest.approx(1.0 - k * k / 1.09, rel=1e-14)
    lml = -0.5 * 0.49 / 1.09 - 0.5 * np.log(1.09) - 0.5 * np.log(2 * np.pi)
    assert gp.log_marginal() == pytest.approx(lml, rel=1e-14)


def test_two_points_explicit_inverse():
    X = np.array([[0.0, 0.0], [1.0, 0.0]])
    y = np.array([1.0, -2.0])
    gp = GP(X, y, hyper=fixed(sigma_n=0.2))
    a = 1.0 + 0.04
    b = np.exp(-0.5)
    Cinv = np.array([[a, -b], [-b, a]]) / (a * a - b * b)
    xs = np.array([0.5, 0.5])
    ks = np.exp(-0.5 * np.array([0.25 + 0.25, 0.25 + 0.25]))
    m, v = gp.predict(xs[None])
    assert m[0] == pytest.approx(ks @ Cinv @ y, rel=1e-13)
    assert v[0] == pytest.approx(1.0 - ks @ Cinv @ ks, rel=1e-13)


def test_noise_free_limit_interpolates():
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 4, (6, 2))
    y = rng.normal(size=6)
    gp = GP(X, y, hyper=fixed(sigma_n=1e-7))
    m, v = gp.predict(X)
    np.testing.assert_allclose(m, y, atol=1e-6)
    assert np.all(np.abs(v) < 1e-6)


def test_far_field_returns_prior():
    gp = GP([[0.0, 0.0], [1.0, 1.0]], [0.5, 0.8], hyper=fixed(sigma_f=1.3))
    m, v = gp.predict([[500.0, -400.0]])
    assert abs(m[0]) < 1e-300 and v[0] == pytest.approx(1.69, rel=1e-12)


def test_mean_separation_by_hand():
    X = np.array([[0.0, 0.0], [1.0, 10.0], [3.0, 20.0]])
    np.testing.assert_allclose(mean_separation(X, (16.0, 0.05), 0), [2.0, 40.0 / 3.0])
    # fewer than two points, or identical inputs: a quarter of the range
    np.testing.assert_allclose(mean_separation(X[:1], (16.0, 0.05), 0), [4.0, 0.0125])
    np.testing.assert_allclose(mean_separation(np.zeros((3, 2)), (16.0, 0.05), 0), [4.0, 0.0125])


def test_posterior_against_explicit_inverse_and_mvn_logpdf():
    rng = np.random.default_rng(2)
    X = rng.uniform([4, 0.001], [20, 0.05], (12, 2))
    y = 0.02 * X[:, 0] ** 2 * X[:, 1] + rng.normal(0, 0.01, 12)
    se = np.full(12, 0.01)
    gp = GP(X, y, se, Hyper())
    # rebuild the same covariance independently
    sc = gp.scale
    D = (X[:, None, :] - X[None, :, :]) / sc
    K = np.exp(-0.5 * (D ** 2).sum(-1))
    C = K + gp.sigma_n ** 2 * np.eye(12)
    Xs = rng.uniform([4, 0.001], [20, 0.05], (5, 2))
    Ds = (Xs[:, None, :] - X[None, :, :]) / sc
    Ks = np.exp(-0.5 * (Ds ** 2).sum(-1))
    Ci = np.linalg.inv(C)
    m, v = gp.predict(Xs)
    np.testing.assert_allclose(m, gp.s_q * Ks @ Ci @ (y / gp.s_q), rtol=1e-9)
    np.testing.assert_allclose(v, gp.s_q ** 2 * (1.0 - np.einsum("ij,jk,ik->i", Ks, Ci, Ks)), rtol=1e-8)
    lml = multivariate_normal(mean=np.zeros(12), cov=C).logpdf(y / gp.s_q)
    assert gp.log_marginal() == pytest.approx(lml, rel=1e-10)
    # the default noise level is the mean standard error, in scaled units
    assert gp.sigma_n == pytest.approx(0.01 / np.sqrt(np.mean(y ** 2)))


def test_append_equals_refit():
    rng = np.random.default_rng(3)
    X = rng.uniform([4, 0.001], [20, 0.05], (8, 2))
    y = rng.normal(size=8)
    se = rng.uniform(0.01, 0.02, 8)
    a = GP(X[:5], y[:5], se[:5])
    for k in range(5, 8):
        a.append(X[k], y[k], se[k])
    b = GP(X, y, se)
    Xs = rng.uniform([4, 0.001], [20, 0.05], (4, 2))
    np.testing.assert_allclose(a.predict(Xs), b.predict(Xs), rtol=1e-12)


def test_interpolation_is_more_certain_than_extrapolation():
    X = np.array([[4.0, 0.01], [8.0, 0.01], [12.0, 0.01]])
    gp = GP(X, [0.1, 0.2, 0.3], [0.01] * 3)
    _, v = gp.predict([[6.0, 0.01], [30.0, 0.01]])
    assert v[0] < v[1]


# ---------------------------------------------------------------- NEXT-4 options
def test_heteroscedastic_noise_is_the_mvn_with_per_point_variances():
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 4, (12, 2))
    y = np.sin(X[:, 0]) + 0.1 * rng.standard_normal(12)
    se = rng.uniform(0.01, 0.3, 12)
    h = fixed(sigma_n=-1.0)
    h.noise_mode = 1
    gp = GP(X, y, se, h)
    # Eq. covarianceEq with each point's own variance, built by a double loop
    C = np.zeros((12, 12))
    for i in range(12):
        for j in range(12):
            d2 = np.sum((X[i] - X[j]) ** 2)  # ranges 4 -> scale 1
            C[i, j] = np.exp(-0.5 * d2) + (se[i] ** 2 if i == j else 0.0)
    assert gp.log_marginal() == pytest.approx(multivariate_normal(np.zeros(12), C).logpdf(y), rel=1e-12)
    # equal SEs reduce it to the uniform-noise GP
    h2 = fixed(sigma_n=0.2)
    gp_u = GP(X, y, None, h2)
    h3 = fixed(sigma_n=-1.0)
    h3.noise_mode = 1
    gp_h = GP(X, y, np.full(12, 0.2), h3)
    xs = rng.uniform(0, 4, (5, 2))
    assert np.allclose(gp_u.predict(xs)[0], gp_h.predict(xs)[0], rtol=1e-12)
    # a point with a huge standard error barely moves the posterior
    se2 = np.full(13, 0.05)
    se2[-1] = 1e4
    X2 = np.vstack([X, [[2.0, 2.0]]])
    y2 = np.append(y, 50.0)
    h4 = fixed(sigma_n=-1.0)
    h4.noise_mode = 1
    gp_big = GP(X2, y2, se2, h4)
    gp_ref = GP(X, y, se2[:12], h4)
    assert np.abs(gp_big.predict(xs)[0] - gp_ref.predict(xs)[0]).max() < 1e-5


def test_periodic_kernel_of_appendix_b():
    T = 10.8
    t = np.linspace(0.0, 30.0, 40)[:, None]
    y = np.sin(2 * np.pi * t[:, 0] / T)
    h = Hyper(sigma_f=1.0, ell=1.0, sigma_n=0.1, out_scale=0, kernel=1, period=T, ranges=(1.0,))
    gp = GP(t, y, None, h)
    K = gp._k(t, t)
    # Eq. periodicKernel, written out: sigma_f^2 exp(-2 sin^2(pi dt / T) / l^2)
    assert K[3, 17] == pytest.approx(np.exp(-2.0 * np.sin(np.pi * abs(t[3, 0] - t[17, 0]) / T) ** 2), rel=1e-14)
    assert gp._k(np.array([[1.0]]), np.array([[1.0 + T]]))[0, 0] == pytest.approx(1.0, abs=1e-14)
    # the posterior mean repeats with the period and follows the sine
    q = np.linspace(5.0, 15.0, 7)[:, None]
    m1, _ = gp.predict(q)
    m2, _ = gp.predict(q + T)
    assert np.allclose(m1, m2, atol=1e-3)
    assert np.abs(m1 - np.sin(2 * np.pi * q[:, 0] / T)).max() < 0.1
    C = K + 0.01 * np.eye(40)
    assert gp.log_marginal() == pytest.approx(multivariate_normal(np.zeros(40), C).logpdf(y), rel=1e-12)


@pytest.mark.parametrize("which", [("sigma_f", "ell"), ("ell", "sigma_n")])
def test_optimised_hyperparameters_maximise_the_evidence(which):
    rng = np.random.default_rng(8)
    X = rng.uniform(0, 4, (30, 2))
    y = np.sin(1.3 * X[:, 0]) * np.cos(0.7 * X[:, 1]) + 0.05 * rng.standard_normal(30)
    gp = GP(X, y, np.full(30, 0.05), fixed(sigma_n=0.1))
    best = gp.optimize(which)
    assert best == pytest.approx(gp.log_marginal(), rel=1e-14)
    theta = {"sigma_f": gp.h.sigma_f, "ell": gp.h.ell, "sigma_n": gp.h.sigma_n}
    # no point of a grid around the optimum does better (a maximum), and the
    # central differences of the evidence vanish there
    for k in which:
        for f in (0.9, 0.97, 1.03, 1.1):
            g2 = GP(X, y, np.full(30, 0.05), fixed(**{**theta, k: theta[k] * f}))
            assert g2.log_marginal() <= best + 1e-9
        e = 1e-4
        up = GP(X, y, None, fixed(**{**theta, k: theta[k] * (1 + e)})).log_marginal()
        dn = GP(X, y, None, fixed(**{**theta, k: theta[k] * (1 - e)})).log_marginal()
        assert abs(up - dn) / (2 * e) < 1e-4


def test_optimised_evidence_is_the_global_maximum_of_a_multimodal_case():
    # a noisy sine under the periodic kernel (App. B): the evidence in
    # (ell, sigma_n) has more than one local maximum (a search from ell = 1
    # alone stops near ell = 1.15).  The optimum is at least the evidence at
    # every point of a fine brute-force grid over the region
    rng = np.random.default_rng(11)
    T = 10.8
    X = np.sort(rng.uniform(0.0, 25.0, 60))[:, None]
    y = np.sin(2 * np.pi * X[:, 0] / T) + 0.15 * rng.standard_normal(60)
    hp = dict(sigma_n=0.3, out_scale=0, kernel=1, period=T, ranges=(1.0,))
    gp = GP(X, y, None, Hyper(**hp))
    best = gp.optimize(("ell", "sigma_n"))
    brute = -np.inf
    for ell in np.exp(np.linspace(np.log(0.3), np.log(6.0), 60)):
        for sn in np.exp(np.linspace(np.log(0.05), np.log(0.5), 40)):
            h = Hyper(**{**hp, "sigma_n": sn})
            h.ell = ell
            brute = max(brute, GP(X, y, None, h).log_marginal())
    assert best >= brute - 1e-9
    assert best > 14.4 and 1.8 < gp.h.ell < 2.6
