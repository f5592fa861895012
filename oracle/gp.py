"""Gaussian-process surrogate oracle, FP64 numpy/scipy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. 2.2-2.3 of the paper:
  - prior f ~ GP(0, K) (Eq. GPEq, zero mean as in Sec. 3.1 / Appendix B);
  - squared-exponential kernel K = sigma_f^2 exp(-d^2 / (2 l^2))
    (Eq. quadraticKernelEq);
  - d^2 = sum_k ((x_ik - x_jk) / mean separation of input k)^2 (Eq. d2Eq),
    the mean separation recomputed whenever the database changes;
  - noisy covariance C = K + sigma_n^2 I (Eq. covarianceEq);
  - posterior mean K(X*, X) C^-1 y (Eq. predMeanEq) and covariance
    K(X*, X*) - K(X*, X) C^-1 K(X, X*) (Eq. predVarEq), whose diagonal is the
    predicted variance that the threshold test uses;
  - log marginal likelihood -1/2 y^T C^-1 y - 1/2 log|C| - n/2 log 2 pi
    (Eq. evidenceEq).
Readings where the paper is silent (also listed in the design notes):
  - "mean separation between inputs" = mean of |x_ik - x_jk| over distinct
    pairs i < j; with fewer than two points, or a zero mean separation, a
    quarter of the stated input range is used;
  - outputs are divided by their RMS before fitting (so sigma_f = 1 is a
    statement in units of the data), and sigma_n, when not given, is the
    mean per-point standard error in the same scaled units (Sec. 2.3 estimates
    sigma_n from the MD data rather than fitting it);
  - the variance compared with the threshold is the latent one (no sigma_n^2).
Options beyond the paper's surrogate:
  - noise_mode 1: heteroscedastic noise, each point's own (SE_i / s_q)^2 on
    the diagonal of C in place of sigma_n^2 (Sec. 2.3 estimates the noise of
    each run from its own data);
  - kernel 1: the periodic kernel of App. B (Eq. periodicKernel) on a single
    input t, K = sigma_f^2 exp(-2 sin^2(pi |t - t'| / T) / l^2), with no
    input normalisation;
  - optimize(): hyperparameters that maximise Eq. evidenceEq (Sec. 2.3, and
    App. B for l and sigma_n of the periodic kernel), found by a library
    optimiser over their logarithms.
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
from scipy.linalg import solve_triangular


@dataclass
class Hyper:
    sigma_f: float = 1.0
    ell: float = 1.0
    sigma_n: float = -1.0          # < 0: mean(y_se) / output scale
    scale_mode: int = 0            # 0 mean pairwise separation, 1 fixed ranges
    ranges: Sequence[float] = field(default_factory=lambda: (16.0, 0.049))
    out_scale: int = 1             # 1: divide outputs by their RMS
    noise_mode: int = 0            # 0 uniform sigma_n, 1 per-point SE_i
    kernel: int = 0                # 0 squared exponential, 1 periodic (App. B)
    period: float = 1.0            # T of the periodic kernel


def mean_separation(X: np.ndarray, ranges, mode: int) -> np.ndarray:
    """Denominators of Eq. d2Eq, one per input."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    fallback = 0.25 * np.asarray(ranges, dtype=np.float64)[:d]
    if mode == 1 or n < 2:
        return fallback.copy()
    out = np.empty(d)
    for k in range(d):
        diffs = np.abs(X[:, None, k] - X[None, :, k])
        iu = np.triu_indices(n, 1)
        m = diffs[iu].mean()
        out[k] = m if m > 0.0 else fallback[k]
    return out


def kernel(A: np.ndarray, B: np.ndarray, scale: np.ndarray, sigma_f: float, ell: float) -> np.ndarray:
    """Eq. quadraticKernelEq on the normalised distance of Eq. d2Eq."""
    D = (A[:, None, :] - B[None, :, :]) / scale[None, None, :]
    d2 = (D ** 2).sum(-1)
    return sigma_f ** 2 * np.exp(-d2 / (2.0 * ell ** 2))


def periodic_kernel(A: np.ndarray, B: np.ndarray, period: float, sigma_f: float, ell: float) -> np.ndarray:
    """Eq. periodicKernel (App. B) on the first input."""
    dt = np.abs(A[:, None, 0] - B[None, :, 0])
    return sigma_f ** 2 * np.exp(-2.0 * np.sin(np.pi * dt / period) ** 2 / ell ** 2)


class GP:
    def __init__(self, X, y, y_se=None, hyper: Optional[Hyper] = None):
        self.h = hyper or Hyper()
        X = np.asarray(X, dtype=np.float64)
        self.X = X.reshape(len(y), X.shape[-1] if X.ndim == 2 else -1)
        self.y = np.asarray(y, dtype=np.float64).copy()
        self.se = np.zeros_like(self.y) if y_se is None else np.asarray(y_se, dtype=np.float64).copy()
        self._fit()

    def _fit(self):
        h = self.h
        n = len(self.y)
        self.scale = mean_separation(self.X, h.ranges, h.scale_mode)
        if h.out_scale and n > 0:
            s = np.sqrt(np.mean(self.y ** 2))
            self.s_q = s if s > 0 else 1.0
        else:
            self.s_q = 1.0
        self.ys = self.y / self.s_q
        self.sigma_n = h.sigma_n / self.s_q if h.sigma_n >= 0 else (self.se.mean() / self.s_q if n else 0.0)
        if n == 0:
            self.L = np.zeros((0, 0))
            self.alpha = np.zeros(0)
            return
        noise = (self.se / self.s_q) ** 2 if h.noise_mode == 1 else np.full(n, self.sigma_n ** 2)
        C = self._k(self.X, self.X) + np.diag(noise)
        self.L = np.linalg.cholesky(C)
        w = solve_triangular(self.L, self.ys, lower=True)
        self.alpha = solve_triangular(self.L.T, w, lower=False)

    def _k(self, A, B):
        h = self.h
        if h.kernel == 1:
            return periodic_kernel(A, B, h.period, h.sigma_f, h.ell)
        return kernel(A, B, self.scale, h.sigma_f, h.ell)

    def append(self, x, y, se=0.0):
        """Alg. 1 database growth: append and update the covariance (the
        normalisation changes with the data, so this refits)."""
        self.X = np.vstack([self.X, np.asarray(x, dtype=np.float64).reshape(1, -1)])
        self.y = np.append(self.y, float(y))
        self.se = np.append(self.se, float(se))
        self._fit()

    def predict(self, Xs):
        """Posterior mean and latent variance in output units."""
        Xs = np.asarray(Xs, dtype=np.float64).reshape(-1, self.X.shape[1])
        sf2 = self.h.sigma_f ** 2
        if len(self.y) == 0:
            return np.zeros(len(Xs)), np.full(len(Xs), sf2 * self.s_q ** 2)
        Ks = self._k(Xs, self.X)
        mean = Ks @ self.alpha
        V = solve_triangular(self.L, Ks.T, lower=True)
        var = sf2 - (V ** 2).sum(0)
        return mean * self.s_q, var * self.s_q ** 2

    def log_marginal(self):
        """Eq. evidenceEq on the scaled outputs."""
        n = len(self.y)
        return float(-0.5 * self.ys @ self.alpha - np.log(np.diag(self.L)).sum() - 0.5 * n * np.log(2 * np.pi))

    def optimize(self, which=("sigma_f", "ell")):
        """Maximise Eq. evidenceEq over the logarithms of the named
        hyperparameters (sigma_n only with uniform noise; it is then held in
        the scaled output units), then refit.  Returns the maximum.

        The evidence can have several local maxima (the periodic kernel's in
        ell does), and the paper asks for the maximising hyperparameters:
        the search evaluates it on a grid of 17 points per hyperparameter over
        two decades either side of the start, then refines by Nelder-Mead
        from the best grid point and from the start, and keeps the larger."""
        from scipy.optimize import minimize
        names = list(which)
        if "sigma_n" in names:
            if self.h.noise_mode == 1:
                raise ValueError("per-point noise has no sigma_n to optimise")
            self.h.sigma_n = self.sigma_n * self.s_q  # hold it explicitly from here on

        def set_theta(t):
            for k, v in zip(names, np.exp(t)):
                if k == "sigma_n":
                    self.h.sigma_n = v * self.s_q
                else:
                    setattr(self.h, k, v)

        def neg(t):
            set_theta(t)
            try:
                self._fit()
            except np.linalg.LinAlgError:
                return 1e300
            return -self.log_marginal()

        t0 = np.log([self.sigma_n if k == "sigma_n" else getattr(self.h, k) for k in names])
        axis = np.log(10.0) * np.linspace(-2.0, 2.0, 17)
        grid = np.stack(np.meshgrid(*([axis] * len(names)), indexing="ij"), -1).reshape(-1, len(names))
        tg = t0 + grid[int(np.argmin([neg(t0 + d) for d in grid]))]
        opts = {"xatol": 1e-10, "fatol": 1e-12, "maxiter": 4000}
        runs = [minimize(neg, t, method="Nelder-Mead", options=opts) for t in (tg, t0)]
        r = min(runs, key=lambda q: q.fun)
        set_theta(r.x)
        self._fit()
        return self.log_marginal()
