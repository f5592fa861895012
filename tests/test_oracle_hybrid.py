"""Pins for the hybrid macro-march oracle (Alg. 1, Eqs. continuityEq and
momentumEq): conservation, threshold limits, Reynolds-lubrication steady
state, closed-form lubrication integral.  CPU only."""
import numpy as np
import pytest

from oracle.gp import GP, Hyper
from oracle.hybrid import Hybrid, HybridCfg, lubrication_integral, poiseuille_flux


class Exact:
    """A surrogate that knows the continuum law exactly (zero spread)."""

    def __init__(self, **kw):
        self.kw = kw

    def predict(self, X):
        return poiseuille_flux(X[:, 0], X[:, 1], **self.kw), np.zeros(len(X))

    def append(self, x, y, se):
        raise AssertionError("an exact surrogate never falls back")


def micro(h, g):
    q = poiseuille_flux(h, g)
    return q, np.full(len(q), 1e-3)


def test_lubrication_integral_closed_form():
    # int (1 + a cos t)^-3 over a period = 2 pi (2 + a^2) / (2 (1 - a^2)^(5/2))
    a = 0.5
    closed = (2 + a * a) / (2 * (1 - a * a) ** 2.5)
    assert closed == pytest.approx(2.3094, abs=1e-4)
    assert lubrication_integral(10.0, a, 2000.0) == pytest.approx(closed * 2000.0 / 1000.0, rel=1e-9)


def test_mass_changes_only_by_boundary_fluxes():
    cfg = HybridCfg(n_sections=50, L=500.0, dt_macro=0.01, tau_rel=1e9)
    hy = Hybrid(cfg, Exact(), micro, var_is_std=True)
    for _ in range(20):
        m0 = hy.mass()
        hy.step()
        q = hy.q
        assert hy.mass() - m0 == pytest.approx(cfg.dt_macro * (q[0] - q[-1]), abs=1e-11 * m0)


def test_threshold_above_signal_gives_zero_flow_without_md():
    # empty database and an absolute threshold above sigma_f (Sec. 3.2): the
    # prior mean (zero) answers every query and no micro-solve runs
    cfg = HybridCfg(n_sections=20, L=200.0, dt_macro=0.01, tau_rel=0.0, tau_abs=1.01)
    hy = Hybrid(cfg, GP(np.zeros((0, 2)), np.zeros(0), None, Hyper()), micro)
    for _ in range(5):
        hy.step()
    assert hy.md_calls == 0 and np.all(hy.q == 0.0)


def test_zero_threshold_calls_md_everywhere():
    cfg = HybridCfg(n_sections=10, L=100.0, dt_macro=0.001, tau_rel=0.0)
    gp = GP(np.zeros((0, 2)), np.zeros(0), None, Hyper())
    hy = Hybrid(cfg, gp, micro)
    for _ in range(3):
        hy.step()
    assert hy.md_calls == 30 and np.all(hy.from_md)


def _steady_flux(n, L=400.0, h0=10.0, dp=2.0, eta=2.0):
    cfg = HybridCfg(n_sections=n, L=L, h0=h0, amp=0.5, dp_mean=dp, dp_amp=0.0, c2=2000.0, tau_rel=1e9)
    # explicit stability: D = c2 rho h^2 / (12 eta) at the widest section
    D = cfg.c2 * 0.8 * (1.5 * h0) ** 2 / (12 * eta)
    cfg.dt_macro = 0.4 * (L / n) ** 2 / D
    hy = Hybrid(cfg, Exact(eta=eta), micro, var_is_std=True)
    for _ in range(int(30000 * (n / 40) ** 2)):
        hy.step()
    return hy.q


def test_steady_state_is_reynolds_lubrication():
    # constant inlet pressure: the march settles to a uniform flux, which
    # converges at first order in the section spacing to the lubrication
    # result Q = rho dp / (12 eta int h^-3 ds)
    q20, q40 = _steady_flux(20), _steady_flux(40)
    # collocated central differences carry a slowly decaying odd-even mode
    assert np.std(q40) < 1e-4 * np.mean(q40)
    Q = 0.8 * 2.0 / (12 * 2.0 * lubrication_integral(10.0, 0.5, 400.0))
    assert np.mean(q40) == pytest.approx(Q, rel=0.05)
    assert 2 * np.mean(q40) - np.mean(q20) == pytest.approx(Q, rel=0.005)


def test_relative_threshold_rule():
    class Stub:
        def predict(self, X):
            return np.array([1.0, -1.0, 0.0, 2.0]), np.array([0.04, 0.06, 0.0, 0.09]) ** 2

        def append(self, x, y, se):
            pass

    cfg = HybridCfg(n_sections=4, L=40.0, dt_macro=1e-4, tau_rel=0.05)
    hy = Hybrid(cfg, Stub(), micro)
    hy.step()
    assert hy.from_md.tolist() == [False, True, False, False]


class Unsure:
    """A surrogate that never answers (unit spread) and learns nothing."""

    def predict(self, X):
        return np.zeros(len(X)), np.ones(len(X))

    def append(self, x, y, se):
        pass


def test_mirror_is_exact_for_an_odd_micro_law():
    # an inlet oscillation strong enough to reverse the flow near the inlet;
    # every query goes to the micro-solver (threshold 0).  The law is odd in
    # g, so answering at |g| with g's sign reproduces the plain march to
    # rounding, and with mirror on the micro-solver never sees g < 0.
    seen = []

    def odd(h, g):
        seen.append(np.min(g))
        return poiseuille_flux(h, g), np.full(len(g), 1e-3)

    kw = dict(n_sections=30, L=300.0, dt_macro=0.004, dp_mean=2.0, dp_amp=3.0, period=20.0, tau_rel=0.0)
    runs = {}
    for mirror in (False, True):
        seen.clear()
        hy = Hybrid(HybridCfg(mirror=mirror, **kw), Unsure(), odd, var_is_std=True)
        negative = False
        for _ in range(60):
            negative |= bool(np.any(hy.forces() < 0.0))
            hy.step()
        runs[mirror] = (hy.rho.copy(), hy.q.copy(), negative, min(seen))
    assert runs[False][2] and runs[False][3] < 0.0  # the flow did reverse somewhere
    assert runs[True][3] >= 0.0
    np.testing.assert_allclose(runs[True][0], runs[False][0], rtol=1e-12)
    np.testing.assert_allclose(runs[True][1], runs[False][1], rtol=1e-10, atol=1e-14)


def test_warm_start_plan_picks_nearest_same_height_run():
    # the oracle march's plan: a section's first fallback starts from the
    # lattice (n_min_cold at least); a later one from the recorded run of the
    # same height with the nearest body force, for its pseudoMD start-up.
    # Heights are compared within a relative 1e-9 (the mirror sections i and
    # n-1-i can differ in the last bit of their cosine)
    from oracle import startup
    cfg = HybridCfg(n_sections=8, L=80.0, h0=10.0, dt_macro=0.002, dp_mean=3.0, dp_amp=0.3, period=6.0,
                    tau_rel=1e-9, warm_start=True, n_min_warm=300, n_min_cold=2500)
    gp = GP(np.zeros((0, 2)), np.zeros(0), None, Hyper(ranges=(16.0, 0.049)))
    hy = Hybrid(cfg, gp, lambda h, g: (poiseuille_flux(h, g), 0.001 + 0.0 * h))
    hy.step()
    assert np.all(hy.plan_prior == -1) and np.all(hy.plan_equil >= 2500)
    hy.step()
    assert len(hy.warm) == 16
    for i in range(8):
        h_i, g_i = hy.warm[8 + i]  # this step's run of section i (all fell back, in order)
        cands = [j for j in range(8) if abs(hy.warm[j][0] - h_i) <= 1e-9 * h_i]
        assert len(cands) >= 1
        # largest covariance = smallest normalised distance (unit scales in
        # the march), ties to the earliest
        best = min(cands, key=lambda j: ((hy.warm[j][0] - h_i) ** 2 + (hy.warm[j][1] - g_i) ** 2, j))
        assert hy.plan_prior[i] == best
        ts = startup.startup_time(h_i, hy.warm[best][1], g_i, 2.5, 0.5, 0.01)
        assert hy.plan_equil[i] == startup.startup_steps(ts, 0.005, 300)
    assert hy.plan_batch_equil == hy.plan_equil.max()


# ---------------------------------------------------------------- the paper's periodic channel
def _paper_cfg(n, **kw):
    base = dict(n_sections=n, L=200.0, h0=10.0, amp=0.2, geometry=1, f_amp=0.03, f_period=4000.0,
                dt_macro=0.05, c2=200.0, tau_rel=1e9)
    base.update(kw)
    return HybridCfg(**base)


def test_paper_geometry_sections_and_heights():
    # Eq. subsEq: s_i = (i - 1) L / N; Eq. heightEq: h = a (cos(2 pi s / L) - 1) + h_1
    hy = Hybrid(_paper_cfg(5), Exact(), micro, var_is_std=True)
    assert np.allclose(hy.s, [0.0, 40.0, 80.0, 120.0, 160.0])
    a = 0.2 * 10.0
    assert hy.h[0] == 10.0 and hy.h.min() == pytest.approx(10.0 - 2 * a * (1 - np.cos(np.pi * 0.8)) / 2, rel=1e-12)
    assert np.allclose(hy.h, a * (np.cos(2 * np.pi * hy.s / 200.0) - 1.0) + 10.0, rtol=0, atol=1e-15)


def test_periodic_channel_conserves_mass_exactly():
    hy = Hybrid(_paper_cfg(40), Exact(), micro, var_is_std=True)
    m0 = hy.mass()
    for _ in range(300):
        hy.step()
    assert hy.mass() == pytest.approx(m0, rel=1e-13)
    assert np.any(hy.q != 0.0)


def test_periodic_channel_reaches_reynolds_lubrication_flow():
    # near the peak of F_ext (quasi-steady: the forcing period is far longer
    # than the pressure relaxation), the flow rate is uniform along the ring
    # and equals Q = F L C / int h^-3 ds with q' = C h^3 g, C = rho^2 / (12 eta);
    # int_0^L (b + a cos(2 pi s / L))^-3 ds = L (2 b^2 + a^2) / (2 (b^2 - a^2)^(5/2)), b = h_1 - a
    n, L, h1, amp = 40, 200.0, 10.0, 0.2
    a = amp * h1
    C = 0.8 ** 2 / (12 * 2.0)
    ds = L / n
    dt = 0.4 * ds * ds / (200.0 * C * h1 ** 3 / (0.8 * h1))  # explicit diffusion limit at the widest section
    cfg = _paper_cfg(n, dt_macro=dt, f_period=40000.0)
    hy = Hybrid(cfg, Exact(), micro, var_is_std=True)
    for _ in range(10000):  # F_ext at sin(pi/2): its peak
        hy.step()
    b = h1 - a
    integral = L * (2 * b * b + a * a) / (2 * (b * b - a * a) ** 2.5)
    Q = 0.03 * L * C / integral
    assert np.abs(hy.q - Q).max() <= 0.002 * Q
    assert hy.q.std() <= 0.001 * Q


def test_forcing_table_replaces_the_sinusoid():
    # Sec. 3.4 forcing variants: step k takes the table's f[k] as F_ext / m.
    # At the first step the densities are uniform, so the pressure gradient
    # vanishes and every section's body force is exactly f[0]: the fluxes are
    # the lubrication law at (h_i, f[0])
    hy = Hybrid(_paper_cfg(10), Exact(), micro, var_is_std=True)
    f = np.array([0.021, -0.004, 0.013])
    hy.set_forcing(f)
    hy.step()
    assert np.array_equal(hy.q, poiseuille_flux(hy.h, np.full(10, 0.021)))
    hy.step()
    hy.step()
    with pytest.raises(ValueError):
        hy.step()  # past the end of the table
    # the sinusoid written out as a table gives the sinusoidal march
    a, b = (Hybrid(_paper_cfg(10, f_period=37.0), Exact(), micro, var_is_std=True) for _ in range(2))
    b.set_forcing(0.03 * np.sin(2.0 * np.pi * np.arange(60) / 37.0))
    for _ in range(60):
        a.step()
        b.step()
        assert np.array_equal(a.q, b.q) and np.array_equal(a.rho, b.rho)
    with pytest.raises(ValueError):
        Hybrid(HybridCfg(n_sections=4), Exact(), micro, var_is_std=True).set_forcing([0.1])


# ---------------------------------------------------------------- pressure surrogate (eos = 1)
class LinearP:
    """A pressure surrogate that is the linear law itself (zero spread)."""

    def __init__(self, X, c2=200.0, rho_ref=0.8, p_out=0.0):
        self.X = np.asarray(X, dtype=np.float64)
        self.c2, self.rho_ref, self.p_out = c2, rho_ref, p_out
        self.appended = []

    def predict(self, X):
        return self.p_out + self.c2 * (X[:, 1] - self.rho_ref), np.zeros(len(X))

    def append(self, x, y, se):
        self.appended.append((float(x[0]), float(x[1]), float(y), float(se)))
        self.X = np.vstack([self.X, np.asarray(x).reshape(1, -1)])


class ThreeInput:
    """A flux surrogate over (h, rho, g) that answers the 2-input law from
    (h, g) and never falls back."""

    def predict(self, X):
        return poiseuille_flux(X[:, 0], X[:, 2]), np.zeros(len(X))

    def append(self, x, y, se):
        raise AssertionError("never falls back")


def test_pressure_surrogate_of_the_linear_law_reproduces_the_linear_march():
    # with p(h, rho) the linear law and a flux law that ignores rho, the
    # eos = 1 march (Alg. 1 with the pressure GP and 3-input flux queries)
    # equals the eos = 0 march to rounding: forces, query and sign plumbing
    kw = dict(n_sections=30, L=300.0, dt_macro=0.004, dp_mean=2.0, dp_amp=0.5, period=20.0, tau_rel=1e9)
    a = Hybrid(HybridCfg(**kw), Exact(), micro, var_is_std=True)
    b = Hybrid(HybridCfg(eos=1, **kw), ThreeInput(), micro, psur=LinearP(np.zeros((0, 2))))
    for _ in range(80):
        a.step()
        b.step()
    np.testing.assert_allclose(b.rho, a.rho, rtol=1e-13)
    np.testing.assert_allclose(b.q, a.q, rtol=1e-11, atol=1e-15)
    b.forces()  # the pressures of the current densities
    np.testing.assert_allclose(b.p, 200.0 * (b.rho - 0.8), rtol=1e-13, atol=1e-13)


def test_fallback_pressures_join_the_pressure_database_once_per_input():
    # Alg. 1: a fallback's pressure is appended when its (h, rho) is not in
    # the pressure database; the pre-simulation inputs count as present
    n = 6
    cfg = HybridCfg(n_sections=n, L=60.0, dt_macro=1e-4, dp_mean=1.0, tau_rel=0.0, eos=1)
    calls = []

    def micro3(h, rho, g):
        calls.append((h.copy(), rho.copy(), g.copy()))
        q = poiseuille_flux(h, g, rho=rho)
        return q, np.full(len(h), 1e-3), 1.5 + 0.0 * h, np.full(len(h), 0.01)

    rho0 = np.linspace(0.81, 0.79, n)  # every (h, rho) distinct (mirrored heights can be equal)
    hy0 = Hybrid(cfg, GP(np.zeros((0, 3)), np.zeros(0), None, Hyper(ranges=(16.0, 0.6, 0.049))), micro3,
                 psur=LinearP(np.zeros((0, 2))), rho0=rho0)
    pre = np.column_stack([hy0.h[:2], hy0.rho[:2]])  # two sections already in the pressure database
    psur = LinearP(pre)
    gp = GP(np.zeros((0, 3)), np.zeros(0), None, Hyper(ranges=(16.0, 0.6, 0.049)))
    hy = Hybrid(cfg, gp, micro3, psur=psur, rho0=rho0)
    hy.step()
    assert len(calls) == 1 and len(calls[0][0]) == n  # threshold 0: every section ran
    np.testing.assert_array_equal(calls[0][1], hy0.rho)  # queried at the sections' own densities
    assert hy.p_appends == n - 2 and len(psur.appended) == n - 2
    assert [(a, b) for a, b, _, _ in psur.appended] == [(float(h), float(r)) for h, r in zip(hy0.h[2:], hy0.rho[2:])]
    assert len(gp.y) == n  # every fallback's flux joined the flux database (3 inputs)
    assert gp.X.shape == (n, 3)
    # a step whose (h, rho) inputs are all present appends no pressure
    before = len(psur.appended)
    hy.rho = hy0.rho.copy()  # back to the first step's densities
    hy.step()
    assert len(psur.appended) == before


def test_presimulation_sweeps_every_distinct_height():
    from oracle.hybrid import presimulate
    seen = []

    def micro_p(h, rho):
        seen.append(len(h))
        return 1.0 + 10.0 * (rho - 0.8) + 0.01 * h, np.full(len(h), 0.003)

    Xp, p, pse = presimulate(micro_p, [10.0, 8.0, 10.0, 6.0], np.linspace(1.0, 0.5, 6))
    assert seen == [18] and Xp.shape == (18, 2)
    assert sorted(set(Xp[:, 0])) == [6.0, 8.0, 10.0]
    np.testing.assert_allclose(p, 1.0 + 10.0 * (Xp[:, 1] - 0.8) + 0.01 * Xp[:, 0])


def test_pressure_database_membership_tolerates_last_bit_differences():
    # the same (h, rho) up to a relative 1e-9 counts as present; a real
    # difference (1e-7) does not
    cfg = HybridCfg(n_sections=4, L=40.0, eos=1)
    hy = Hybrid(cfg, ThreeInput(), micro, psur=LinearP(np.array([[10.0, 0.8], [12.0, 0.75]])))
    assert hy.p_known(np.array([10.0 * (1 + 4e-16), 0.8]))
    assert hy.p_known(np.array([12.0, 0.75 * (1 - 5e-10)]))
    assert not hy.p_known(np.array([10.0, 0.8 * (1 + 1e-7)]))
    assert not hy.p_known(np.array([12.0, 0.8]))
