"""Standard error of a time average from a correlated series (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper (Sec. 2.3, the paragraph on hyperparameters) takes the noise level
of each MD run as the standard deviation of its mean output, computed from the
raw time-instantaneous data.  Successive samples of a flow rate are strongly
correlated (the streamwise momentum of the fluid relaxes through the walls
over a viscous time of order h^2 / nu), so the naive sigma / sqrt(n) is far
too small.  Two estimators are written out here:

``geyer``   the initial monotone sequence estimator of C. J. Geyer,
            "Practical Markov chain Monte Carlo", Statistical Science 7
            (1992) 473-483, Sec. 3.3.  From the empirical autocovariances
            gamma_t = (1/n) sum_{i<n-t} (x_i - mean)(x_{i+t} - mean), the
            pair sums Gamma_k = gamma_{2k} + gamma_{2k+1} are kept while they
            stay positive (initial positive sequence), each replaced by the
            smallest of Gamma_0..Gamma_k (monotone), and the asymptotic
            variance is  -gamma_0 + 2 sum_k Gamma_k.  The variance of the mean
            is that over n.
``blocks``  the standard deviation of nb contiguous equal block means over
            sqrt(nb), a remainder of n mod nb samples dropped from the front.

Readings (where the source is silent):
  * when Gamma_0 is not positive (a strongly anti-correlated series) the
    sequence is empty, and when the sum comes out not positive, the iid
    value gamma_0 / n is returned;
  * the sequence also ends when the pair would reach past lag n - 1.
"""
import numpy as np


def autocovariance(x):
    """gamma_t for t = 0 .. n-1 with the 1/n normalisation (all lags)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x - x.mean()
    # full cross-correlation of d with itself; entry n-1+t is sum_i d_i d_{i+t}
    return np.correlate(d, d, mode="full")[n - 1:] / n


def geyer_variance(x):
    """Asymptotic variance sigma^2 (variance of the mean = sigma^2 / n) and the
    number of pair sums used."""
    return geyer_from_autocovariance(autocovariance(x))


def geyer_from_autocovariance(g):
    """The initial monotone sequence over given autocovariances gamma_0..n-1:
    (sigma^2, number of pair sums used)."""
    g = np.asarray(g, dtype=np.float64)
    n = len(g)
    total, used, smallest = 0.0, 0, np.inf
    k = 0
    while 2 * k + 1 < n:
        gam = g[2 * k] + g[2 * k + 1]
        if not gam > 0.0:
            break
        smallest = min(smallest, gam)
        total += smallest
        used += 1
        k += 1
    var = -g[0] + 2.0 * total if used > 0 else g[0]
    if not var > 0.0:
        var = g[0]
    return float(var), used


def geyer(x):
    """(mean, SE) of the time average of x."""
    x = np.asarray(x, dtype=np.float64)
    var, _ = geyer_variance(x)
    return float(x.mean()), float(np.sqrt(var / len(x)))


def blocks(x, nb):
    """(mean, SE) from nb contiguous block means; remainder dropped in front."""
    x = np.asarray(x, dtype=np.float64)
    B = len(x) // nb
    r = len(x) - nb * B
    bm = x[r:].reshape(nb, B).mean(axis=1)
    return float(bm.mean()), float(bm.std(ddof=1) / np.sqrt(nb))


def halves(x):
    """Means of the first and second half (the second takes the odd sample)."""
    x = np.asarray(x, dtype=np.float64)
    h = len(x) // 2
    return float(x[:h].mean()), float(x[h:].mean())


def ar1_variance_of_mean(phi, sigma_e, n):
    """Exact variance of the mean of n samples of a stationary AR(1) process
    x_t = phi x_{t-1} + e_t, e_t ~ N(0, sigma_e^2):
    Var(mean) = (s^2 / n) [1 + 2 sum_{k=1}^{n-1} (1 - k/n) phi^k],
    s^2 = sigma_e^2 / (1 - phi^2), summed in closed form."""
    s2 = sigma_e * sigma_e / (1.0 - phi * phi)
    # sum_{k=1}^{n-1} (1 - k/n) phi^k
    #   = phi/(1-phi) - phi (1 - phi^n) / (n (1-phi)^2)
    acc = phi / (1.0 - phi) - phi * (1.0 - phi ** n) / (n * (1.0 - phi) ** 2)
    return s2 / n * (1.0 + 2.0 * acc)
