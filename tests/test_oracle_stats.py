"""Pins for the oracle's standard error of a correlated time average.

The estimator (Geyer's initial monotone sequence, Statistical Science 1992,
Sec. 3.3) is checked against a hand computation, brute-force autocovariances,
the exact variance of the mean of an AR(1) process (itself checked against a
direct sum), and its iid limit.  CPU only.
"""
import numpy as np
import pytest

from oracle import stats


def test_hand_computed_four_samples():
    # x = 1, 2, 3, 4: mean 2.5, d = (-1.5, -0.5, 0.5, 1.5);
    # gamma_0 = 5/4, gamma_1 = (0.75 - 0.25 + 0.75)/4 = 0.3125,
    # gamma_2 = (-0.75 - 0.75)/4 = -0.375, gamma_3 = -2.25/4 = -0.5625.
    # Gamma_0 = 1.5625 > 0, Gamma_1 = -0.9375 ends the sequence:
    # sigma^2 = -1.25 + 2 * 1.5625 = 1.875, SE = sqrt(1.875 / 4).
    g = stats.autocovariance([1.0, 2.0, 3.0, 4.0])
    assert np.allclose(g, [1.25, 0.3125, -0.375, -0.5625], rtol=0, atol=1e-15)
    var, used = stats.geyer_variance([1.0, 2.0, 3.0, 4.0])
    assert used == 1 and var == pytest.approx(1.875, abs=1e-15)
    m, se = stats.geyer([1.0, 2.0, 3.0, 4.0])
    assert m == 2.5 and se == pytest.approx(np.sqrt(1.875 / 4.0), rel=1e-15)


def test_monotone_step_takes_the_running_minimum():
    # hand-made autocovariances: Gamma = (0.4, 0.8, 0.3, -0.7).  The positive
    # sequence ends before Gamma_3; the monotone one replaces Gamma_1 by
    # Gamma_0: sigma^2 = -1 + 2 (0.4 + 0.4 + 0.3) = 1.2 (without the
    # replacement it would be 2.0)
    g = [1.0, -0.6, 0.5, 0.3, 0.2, 0.1, -0.5, -0.2]
    var, used = stats.geyer_from_autocovariance(g)
    assert used == 3
    assert var == pytest.approx(1.2, abs=1e-15)


def test_alternating_series_falls_back_to_iid():
    # x = (1, -1, 1, -1, ...) has gamma_t = (-1)^t (1 - t/n), so every pair
    # sum is 1/n > 0 and all n/2 are kept: sigma^2 = -1 + 2 (n/2)(1/n) = 0,
    # not positive, and the iid value gamma_0 = 1 is used
    n = 64
    x = np.tile([1.0, -1.0], n // 2)
    g = stats.autocovariance(x)
    t = np.arange(n)
    assert np.allclose(g, (-1.0) ** t * (1.0 - t / n), atol=1e-14)
    var, used = stats.geyer_variance(x)
    assert used == n // 2
    assert var == pytest.approx(1.0)


def test_autocovariance_equals_brute_force():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(301)
    d = x - x.mean()
    brute = np.array([sum(d[i] * d[i + t] for i in range(len(x) - t)) / len(x) for t in range(len(x))])
    assert np.allclose(stats.autocovariance(x), brute, rtol=0, atol=1e-13)


def test_ar1_closed_form_equals_direct_sum():
    for phi, n in [(0.0, 10), (0.5, 7), (0.9, 200), (-0.3, 33)]:
        s2 = 1.0 / (1.0 - phi * phi)
        direct = s2 / n * (1.0 + 2.0 * sum((1.0 - k / n) * phi ** k for k in range(1, n)))
        assert stats.ar1_variance_of_mean(phi, 1.0, n) == pytest.approx(direct, rel=1e-12)


def _ar1(rng, phi, n, reps):
    e = rng.standard_normal((reps, n))
    x = np.empty_like(e)
    x[:, 0] = e[:, 0] / np.sqrt(1.0 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return x


@pytest.mark.parametrize("phi", [0.0, 0.9, 0.98])
def test_geyer_is_calibrated_on_ar1(phi):
    # integrated autocorrelation times 0.5, 9.5 and 49.5 samples over n = 4000:
    # the mean of SE^2 over replicates matches the exact variance of the mean
    # within the replicate noise, and 2 SE covers close to 95 %
    rng = np.random.default_rng(int(phi * 100) + 1)
    n, reps = 4000, 300
    x = _ar1(rng, phi, n, reps)
    exact = stats.ar1_variance_of_mean(phi, 1.0, n)
    se = np.array([stats.geyer(r)[1] for r in x])
    assert np.mean(se ** 2) == pytest.approx(exact, rel=0.12)
    cover = np.mean(np.abs(x.mean(axis=1)) <= 2.0 * se)
    assert 0.90 <= cover <= 0.99
    if phi <= 0.9:
        # the block rule with 20 blocks of 200 samples is also fine where the
        # blocks are twenty correlation times long (at phi = 0.98, only four)
        se_b = np.array([stats.blocks(r, 20)[1] for r in x])
        assert np.mean(se_b ** 2) == pytest.approx(exact, rel=0.2)


def test_geyer_sees_correlations_the_block_rule_misses():
    # correlation time of 500 samples against blocks of 200: the 20-block
    # rule underestimates the variance of the mean, Geyer's estimator much less
    rng = np.random.default_rng(3)
    phi = (2 * 500 - 1) / (2 * 500 + 1)
    n, reps = 4000, 200
    x = _ar1(rng, phi, n, reps)
    exact = stats.ar1_variance_of_mean(phi, 1.0, n)
    geyer = np.mean([stats.geyer(r)[1] ** 2 for r in x])
    block = np.mean([stats.blocks(r, 20)[1] ** 2 for r in x])
    assert block < 0.5 * exact
    assert geyer > 1.3 * block


def test_iid_limit():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(20000)
    m, se = stats.geyer(x)
    assert se == pytest.approx(x.std() / np.sqrt(len(x)), rel=0.1)


def test_blocks_and_halves():
    x = np.arange(1.0, 24.0)  # 23 samples: 20 blocks of 1 after dropping 3 in front
    m, se = stats.blocks(x, 20)
    assert m == pytest.approx(np.mean(np.arange(4.0, 24.0)))
    assert se == pytest.approx(np.std(np.arange(4.0, 24.0), ddof=1) / np.sqrt(20))
    assert stats.halves([1.0, 2.0, 3.0]) == (1.0, 2.5)
