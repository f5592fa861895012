"""Pins for the oracle's flow observables: the sampled mass flow rate per unit
span against the mass that crosses a cross-section, the x-momentum balance of
velocity Verlet with the body force of Eq. momentumEq, and the steady force
balance between body force and walls.  CPU only.

The flow rate q' = sum(m v_x) / (Lx Lz) (Sec. 2.1) is compared with a second
definition that shares none of its arithmetic: the net number of atoms that
cross the periodic plane x = 0, per unit time and unit span.  For atom i with
start x0_i and unwrapped displacement D_i its net crossings are
floor((x0_i + D_i) / Lx), so

    crossings Lx = sum D_i + sum x0_i - sum x_end_i,

and velocity Verlet moves each atom by dt times its half-step velocity, so

    sum D_i = dt [sum_samples P - P_end + P_start + dt/2 K1],

with P = sum v_x after a step and K1 the summed x kick force (pair force plus
body force) of the first half-kicks of the sampled steps.  The crossing rate
therefore equals the time average of q' up to two boundary terms that decay
as 1/T.
"""
import numpy as np
import pytest

from oracle import md, stats

SMALL = dict(Lx_nom=12.0, Lz_nom=12.0)


@pytest.fixture(scope="module")
def driven_channel():
    # h = 6 channel of the literal 12 x 12 box, strong drive g = 0.15:
    # 2000 start-up steps, then 10,000 sampled steps
    p = md.Params(n_equil=2000, **SMALL)
    s = md.System(6.0, 0.15, 5, p)
    s.run(2000)
    x0, _ = s.get_state()
    s.run(10000)
    return s, p, x0


def test_mass_crossing_a_section_is_the_flux(driven_channel):
    s, p, x0 = driven_channel
    d = s.flow_diag()
    x1, _ = s.get_state()
    disp = s.displacements()
    ns = int(d["samples"])
    assert ns == 10000
    T = ns * p.dt
    # net crossings of x = 0, atom by atom, from start position and displacement
    per_atom = np.floor((x0[:, 0] + disp) / s.Lx)
    assert d["wraps"] == per_atom.sum()
    # crossings Lx = sum D + sum x0 - sum x_end (each wrap moves an atom by Lx)
    assert d["wraps"] * s.Lx == pytest.approx(disp.sum() + x0[:, 0].sum() - x1[:, 0].sum(), abs=1e-7)
    # sum D = dt [sum_samples P - P_end + P_start + dt/2 K1]
    q = s.series()
    A = s.Lx * s.Lz
    P_sum = q.sum() * A
    rhs = p.dt * (P_sum - d["p_now"] + d["p_start"] + 0.5 * p.dt * d["kick1"])
    assert disp.sum() == pytest.approx(rhs, rel=1e-10)
    # the crossing rate per unit span against the sampled flux: equal up to
    # the two boundary terms, which decay as 1/T.  b2 is the change of the
    # summed positions inside the cell over the window: for N atoms spread
    # uniformly over [0, Lx) at both ends its standard deviation is
    # Lx sqrt(N / 6) / (Lx Lz T)
    q_cross = d["wraps"] / (s.Lz * T)
    q_mean = q.mean()
    b1 = (d["p_start"] - d["p_now"] + 0.5 * p.dt * d["kick1"]) / (A * ns)
    b2 = (x0[:, 0].sum() - x1[:, 0].sum()) / (s.Lx * s.Lz * T)
    assert q_cross == pytest.approx(q_mean + b1 + b2, rel=1e-9)
    assert q_mean > 0.0
    assert abs(b1) < 0.01 * q_mean
    assert abs(b2) <= 3.0 * np.sqrt(s.n_fluid / 6.0) / (s.Lz * T)
    assert abs(q_cross - q_mean) < 0.5 * q_mean
    assert s.result()["flux"] == q_mean


def test_x_momentum_balance(driven_channel):
    # Eq. momentumEq: every fluid atom carries m g along +x; the thermostat
    # acts on y only; fluid-fluid forces cancel pairwise.  Velocity Verlet
    # then changes sum m v_x by exactly dt/2 (K1 + K2) over the window.
    s, p, _ = driven_channel
    d = s.flow_diag()
    assert d["p_now"] - d["p_start"] == pytest.approx(0.5 * p.dt * (d["kick1"] + d["kick2"]), abs=1e-8)
    # the summed pair force is the wall force: the fluid-fluid part cancels
    assert d["fpair_x"] == pytest.approx(d["fwall_x"], abs=1e-8 * abs(d["fwall_x"]) + 1e-8)
    # K2 sums pair plus body force over the sampled steps: N g per step enters
    ns = int(d["samples"])
    assert d["kick2"] == pytest.approx(d["fpair_x"] + ns * s.n_fluid * s.g, rel=1e-10)


def test_walls_balance_the_body_force(driven_channel):
    # steady state: the walls hold the fluid against the body force,
    # <F_wall,x> = -N_f m g, within two standard errors of the wall-force
    # time average (Geyer's estimator over its per-step series)
    s, p, _ = driven_channel
    fw = s.wall_force_series()
    m, se = stats.geyer(fw)
    target = -s.n_fluid * s.g
    assert m < 0.0
    assert abs(m - target) <= 2.0 * se, (m, target, se)
    assert se < 0.1 * abs(target)  # the check is not vacuous
    # each wall takes its share along y too: at rest in y the two walls push
    # the fluid with equal and opposite normal forces
    d = s.flow_diag()
    assert d["fwall_y_lo"] > 0.0 and d["fwall_y_hi"] < 0.0
    assert d["fwall_y_lo"] == pytest.approx(-d["fwall_y_hi"], rel=0.05)


def test_pressure_series_is_the_wall_normal_force_per_area():
    # per sampled step the mean of the two walls' normal forces on the fluid
    # per unit area; its mean is the summed wall forces over the samples, and
    # the two walls push with equal and opposite mean force at rest
    p = md.Params(n_equil=500, Lx_nom=12.0, Lz_nom=12.0)
    s = md.System(7.0, 0.0, 4, p)
    s.run(2500)
    d = s.flow_diag()
    ps = s.pressure_series()
    assert len(ps) == 2000 == d["samples"]
    assert ps.mean() == pytest.approx(0.5 * (d["fwall_y_lo"] - d["fwall_y_hi"]) / 2000 / (s.Lx * s.Lz), rel=1e-12)
    r = s.result()
    assert r["p"] == pytest.approx(ps.mean(), rel=1e-12) and 0.0 < r["p_se"] < 0.1 * r["p"]
    assert d["fwall_y_lo"] == pytest.approx(-d["fwall_y_hi"], rel=0.05)
