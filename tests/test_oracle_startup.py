"""Pins for the warm-start oracle (Alg. 1 "find nearest prior input" and
"pseudoMD"; Sec. 2.4): the slip eigenvalues against their closed form and
their defining equation, the modal flow-rate deviation at t = 0 against the
two steady profiles, the start-up time against an independent explicit
finite-difference solve of the same 1-D problem, its h^2 scaling, and the
prior selection against brute force.  CPU only."""
import numpy as np
import pytest

from oracle import startup as su


def test_no_slip_eigenvalues_are_odd_half_waves():
    k = su.eigen_k(10.0, 0.0, 5)
    assert np.allclose(k, (2 * np.arange(1, 6) - 1) * np.pi / 10.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("b", [0.3, 1.0, 5.0])
def test_slip_eigenvalues_solve_their_equation(b):
    h = 8.0
    k = su.eigen_k(h, b, 30)
    z = k * h / 2.0
    assert np.all(np.abs(np.cos(z) - b * k * np.sin(z)) < 1e-13 * (1.0 + b * k))
    assert np.all(np.diff(k) > 0)
    # the first root lies below the no-slip one: slip lets the flow relax slower
    assert k[0] < np.pi / h


@pytest.mark.parametrize("b", [0.0, 0.5])
def test_initial_deviation_is_the_difference_of_steady_flow_rates(b):
    h, nu = 12.0, 2.5
    cw, rate = su.deviation_modes(h, 0.013, nu, b, n_modes=400)
    assert cw.sum() == pytest.approx(su.flow_rate(h, 0.013, nu, b), rel=1e-7)
    assert np.all(rate > 0)


def _fd_startup(h, g_in, g_new, nu, b, tol, M=100):
    # explicit finite differences on M cells, ghost cells carrying the slip
    # condition u_wall = b du/dn at both walls
    dy = h / M
    y = (np.arange(M) + 0.5) * dy
    u = (g_in / (2 * nu)) * (y * (h - y) + b * h)
    q_new = su.flow_rate(h, g_new, nu, b)
    scale = max(abs(q_new), abs(su.flow_rate(h, g_in, nu, b)))
    dt = 0.2 * dy * dy / nu
    f = (2 * b - dy) / (2 * b + dy)
    t = 0.0
    while abs(u.sum() * dy - q_new) > tol * scale:
        ul = np.concatenate([[f * u[0]], u[:-1]])
        ur = np.concatenate([u[1:], [f * u[-1]]])
        u = u + dt * (g_new + nu * (ul - 2 * u + ur) / (dy * dy))
        t += dt
    return t


@pytest.mark.parametrize("h,g_in,g_new,b", [(10.0, 0.0, 0.02, 0.0), (10.0, 0.0, 0.02, 0.5),
                                            (6.0, 0.03, 0.02, 0.5), (15.0, 0.01, 0.012, 1.0)])
def test_startup_time_matches_a_finite_difference_solve(h, g_in, g_new, b):
    nu, tol = 2.5, 0.01
    ts = su.startup_time(h, g_in, g_new, nu, b, tol)
    assert ts == pytest.approx(_fd_startup(h, g_in, g_new, nu, b, tol), rel=0.02)


def test_startup_time_scales_with_h_squared_and_vanishes_near_the_target():
    nu, tol = 2.5, 0.01
    t1 = su.startup_time(8.0, 0.0, 0.02, nu, 0.0, tol)
    t2 = su.startup_time(16.0, 0.0, 0.02, nu, 0.0, tol)
    assert t2 == pytest.approx(4.0 * t1, rel=1e-9)
    # a prior within the tolerance needs no start-up
    assert su.startup_time(8.0, 0.02 * 1.005, 0.02, nu, 0.0, tol) == 0.0
    # starting from rest, the tolerance is relative to the new flow alone
    t_rest = su.startup_time(8.0, 0.0, 0.02, nu, 0.0, tol)
    assert t_rest == pytest.approx(su.startup_time(8.0, 0.0, 0.002, nu, 0.0, tol), rel=1e-9)
    # a start-up never takes longer than the one from rest to the larger flow
    assert su.startup_time(8.0, 0.01, 0.012, nu, 0.0, tol) < su.startup_time(8.0, 0.0, 0.012, nu, 0.0, tol)
    # the closer the prior, the shorter the start-up
    assert su.startup_time(8.0, 0.018, 0.02, nu, 0.0, tol) < su.startup_time(8.0, 0.01, 0.02, nu, 0.0, tol)
    assert su.startup_steps(1.234, 0.005, 100) == 247
    assert su.startup_steps(0.1, 0.005, 100) == 100


def test_nearest_prior_is_brute_force_over_same_height_entries():
    rng = np.random.default_rng(4)
    hs = np.array([5.0, 7.5, 10.0])
    X = np.column_stack([rng.choice(hs, 40), rng.uniform(0.001, 0.05, 40)])
    has = rng.uniform(size=40) < 0.8
    scale = np.array([2.0, 0.01])
    for _ in range(20):
        x = np.array([rng.choice(hs), rng.uniform(0.001, 0.05)])
        i = su.nearest_prior(X, x, scale, has)
        cand = [j for j in range(40) if has[j] and X[j, 0] == x[0]]
        if not cand:
            assert i == -1
            continue
        kern = [np.exp(-0.5 * np.sum(((X[j] - x) / scale) ** 2)) for j in cand]
        assert i == cand[int(np.argmax(kern))]
    assert su.nearest_prior(X, np.array([6.0, 0.01]), scale, has) == -1
