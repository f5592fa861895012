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
