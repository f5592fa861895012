"""Warm starts of fallback MD runs (Alg. 1, "find nearest prior input" and
"pseudoMD"; Sec. 2.4), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A new MD run starts from the final state of the database entry whose input
maximises the covariance K(x_in, x*) with the new input, among entries of the
same channel height (the atom count depends on h); with no such entry it
starts from the lattice at rest.  Its start-up phase t_s comes from a 1-D
Navier-Stokes solve of the channel with a Navier slip condition:

    du/dt = g* + nu d2u/dy2 on 0 < y < h,   u = b du/dn at both walls,

started from the steady profile of the prior input's body force g_in (rest:
g_in = 0), u_g(y) = (g / 2 nu) [y (h - y) + b h].  The deviation from the
new steady profile decays in the symmetric modes cos(k_n (y - h/2)) with
cot(k_n h / 2) = b k_n; t_s is the first time at which the flow rate is
within `tol` of its new steady value, relative to the larger of the two
steady flow rates: |q(t) - q*| <= tol max(|q_in|, |q*|).

Readings (where the paper is silent): the slip length b and kinematic
viscosity nu are model constants; the tolerance is relative to the larger of
the old and new steady flow rates (a start-up between two nearly equal, or
two nearly zero, flows is short); a run never equilibrates for less than a
stated minimum (thermal relaxation; longer from the lattice than from a
stored state).
"""
import numpy as np


def eigen_k(h, b, n_modes):
    """First n_modes roots of cot(k h / 2) = b k (k_n h / 2 in ((n-1) pi,
    (n - 1/2) pi]), by bisection to full precision."""
    ks = np.zeros(n_modes)
    for n in range(1, n_modes + 1):
        lo, hi = (n - 1) * np.pi, (n - 0.5) * np.pi  # in z = k h / 2
        if b == 0.0:
            ks[n - 1] = 2.0 * hi / h
            continue
        # f(z) = cos z - (2 b / h) z sin z: positive just above lo, <= 0 at hi
        c = 2.0 * b / h
        a = lo + 1e-15 if n == 1 else lo
        fa = np.cos(a) - c * a * np.sin(a)
        for _ in range(200):
            m = 0.5 * (a + hi)
            fm = np.cos(m) - c * m * np.sin(m)
            if (fm > 0.0) == (fa > 0.0):
                a, fa = m, fm
            else:
                hi = m
        ks[n - 1] = 2.0 * (0.5 * (a + hi)) / h
    return ks


def flow_rate(h, g, nu, b):
    """Steady flow rate per unit span per unit density: int u_g dy =
    g h^3 (1 + 6 b / h) / (12 nu)."""
    return g * h ** 3 * (1.0 + 6.0 * b / h) / (12.0 * nu)


def deviation_modes(h, dg, nu, b, n_modes=200):
    """Modal weights c_n and rates r_n of the flow-rate deviation
    Q(t) = sum_n c_n exp(-r_n t) for an initial profile that differs from the
    steady one by the steady profile of body force dg."""
    k = eigen_k(h, b, n_modes)
    a = 0.5 * h
    s, c = np.sin(k * a), np.cos(k * a)
    phi_int = 2.0 * s / k                        # int cos(k X) dX over [-a, a]
    phi_sq = a + np.sin(2.0 * k * a) / (2.0 * k)  # int cos^2(k X) dX
    x2 = 2.0 * a * a * s / k + 4.0 * a * c / k ** 2 - 4.0 * s / k ** 3  # int X^2 cos(k X) dX
    w0_proj = (dg / (2.0 * nu)) * ((a * a + b * h) * phi_int - x2)  # int w0 cos(k X) dX
    coef = w0_proj / phi_sq
    return coef * phi_int, nu * k * k


def startup_time(h, g_in, g_new, nu, b, tol, n_modes=200):
    """t_s: the first t >= 0 with |q(t) - q*| <= tol max(|q_in|, |q*|)
    (bisection on the modal sum, monotone once its first mode dominates)."""
    q_new = flow_rate(h, g_new, nu, b)
    q_in = flow_rate(h, g_in, nu, b)
    cw, rate = deviation_modes(h, g_in - g_new, nu, b, n_modes)

    def dev(t):
        return abs(float(np.sum(cw * np.exp(-rate * t))))

    target = tol * max(abs(q_in), abs(q_new))
    if dev(0.0) <= target:
        return 0.0
    hi = 1.0 / rate[0]
    while dev(hi) > target:
        hi *= 2.0
    lo = 0.0
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if dev(m) > target:
            lo = m
        else:
            hi = m
    return hi


def startup_steps(t_s, dt, n_min):
    """Equilibration steps of a run: ceil(t_s / dt), at least n_min."""
    return max(int(n_min), int(np.ceil(t_s / dt - 1e-9)))


def nearest_prior(X_db, x_star, scale, has_state):
    """Index of the database entry with a stored state, the same channel
    height as x_star (first input; equal within a relative 1e-9, since
    heights computed with different libraries' cosines can differ in the
    last bits), and the largest squared-exponential covariance with x_star
    over inputs normalised by `scale` (Eq. quadraticKernelEq: the smallest
    normalised distance); -1 when none.  Ties go to the earliest entry."""
    best, best_d = -1, np.inf
    for i, x in enumerate(np.asarray(X_db, dtype=np.float64)):
        if not has_state[i] or abs(x[0] - x_star[0]) > 1e-9 * max(abs(x[0]), abs(x_star[0])):
            continue
        d = float(np.sum(((x - x_star) / scale) ** 2))
        if d < best_d:
            best, best_d = i, d
    return best
