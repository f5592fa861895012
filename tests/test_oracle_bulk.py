"""Pins for the oracle's bulk periodic box: the virial of a pair against its
closed form, momentum conservation, and two cross-checks of the channel
against the bulk liquid at the channel's own core density:

* shear viscosity from the curvature of the Poiseuille profile of a wide
  channel (Sec. 2.1: the subdomain flow is pressure- or body-force-driven
  channel flow) against the periodic sinusoidal-force method (Gosling,
  McDonald & Singer, Mol. Phys. 26 (1973) 1475: a body force g0 sin(k y)
  gives the steady profile u(y) = rho g0 sin(k y) / (eta k^2));
* the normal force per unit area that the fluid exerts on a wall against
  the virial pressure rho T + W / (3 V) of the bulk liquid (the yy momentum
  balance makes P_yy uniform across the channel).

CPU only.
"""
import numpy as np
import pytest

from oracle import md

BOX = dict(Lx_nom=12.0, Lz_nom=12.0)


def _bulk(rho, n_equil, seed=1, g_sin=0.0, h=12.699):
    p = md.Params(wall_layers=0, periodic_y=1, rho=rho, n_equil=n_equil, g_sin=g_sin, bin_dy=h / 40.0, **BOX)
    return md.System(h, 0.0, seed, p), p


def test_virial_of_two_atoms():
    # W = r . f(r) = 24 (2 r^-12 - r^-6) for one pair at separation r; here
    # the pair straddles the periodic boundary in y
    p = md.Params(wall_layers=0, periodic_y=1, n_fluid=2, **BOX)
    s = md.System(12.699, 0.0, 1, p)
    r = 1.2
    x = np.array([[2.0, 0.5, 2.0], [2.0, 0.5 - r + s.h, 2.0]])
    s.set_state(x, np.zeros((2, 3)))
    fd = s.force_diag()
    w = 24.0 * (2.0 * r ** -12 - r ** -6)
    assert fd["virial"] == pytest.approx(w, rel=1e-12)
    assert fd["virial_yy"] == pytest.approx(w, rel=1e-12)  # separation along y only
    f, _ = s.forces_cells()
    assert f[0, 1] == pytest.approx(w / r, rel=1e-12)  # repulsive: atom 0 pushed to +y
    assert f[1, 1] == pytest.approx(-w / r, rel=1e-12)


def test_bulk_box_forces_and_momentum():
    s, p = _bulk(0.8, 0)
    s.run(50)
    f, _ = s.forces_cells()
    fb, _ = s.forces_brute()
    assert np.abs(f - fb).max() <= 1e-12 * max(1.0, np.abs(fb).max())
    assert np.abs(f.sum(axis=0)).max() <= 1e-10 * np.abs(f).sum()
    # NVE in the bulk box: total momentum stays constant
    _, v0 = s.get_state()
    s.run(200, thermostat=False)
    _, v1 = s.get_state()
    assert np.abs(v1.sum(axis=0) - v0.sum(axis=0)).max() <= 1e-9


@pytest.fixture(scope="module")
def wide_channel():
    # h = 20, g = 0.02, thermostat on z (v_z), 12,000 start-up + 36,000
    # sampled steps
    p = md.Params(n_equil=12000, thermo_axis=2, **BOX)
    s = md.System(20.0, 0.02, 3, p)
    s.run(48000)
    return s, p


@pytest.mark.slow
def test_channel_viscosity_and_pressure_match_the_bulk_liquid(wide_channel):
    s, p = wide_channel
    g = s.g
    mvx, cnt = s.profile()
    y = (np.arange(len(mvx)) + 0.5) * p.bin_dy
    u = mvx / np.maximum(cnt, 1.0)
    core = (y > 3.0) & (y < 17.0)
    rho_core = cnt[core].sum() / cnt.sum() * s.n_fluid / (s.Lx * s.Lz * core.sum() * p.bin_dy)
    A = np.column_stack([np.ones(core.sum()), y[core], y[core] ** 2])
    c, *_ = np.linalg.lstsq(A, u[core], rcond=None)
    fit = A @ c
    r2 = 1.0 - np.sum((u[core] - fit) ** 2) / np.sum((u[core] - u[core].mean()) ** 2)
    assert r2 >= 0.98
    assert abs(-c[1] / (2.0 * c[2]) - 10.0) < 0.5  # vertex at the mid-plane
    eta_curv = -rho_core * g / (2.0 * c[2])

    # bulk liquid at the core density: sinusoidal force of amplitude 0.1
    b, pb = _bulk(round(rho_core, 4), 3000, g_sin=0.1)
    b.run(3000 + 20000)
    mb, cb = b.profile()
    yb = (np.arange(len(mb)) + 0.5) * pb.bin_dy
    ub = mb / np.maximum(cb, 1.0)
    k = 2.0 * np.pi / b.h
    cs, *_ = np.linalg.lstsq(np.column_stack([np.sin(k * yb), np.cos(k * yb), np.ones_like(yb)]), ub, rcond=None)
    rho_b = b.n_fluid / (b.Lx * b.Lz * b.h)
    eta_sin = rho_b * 0.1 / (k * k * cs[0])
    assert abs(cs[1]) < 0.1 * cs[0]  # in phase with the force
    assert eta_curv == pytest.approx(eta_sin, rel=0.10), (eta_curv, eta_sin, rho_core)

    # normal pressure on the walls against the bulk virial pressure
    d = s.flow_diag()
    n = d["samples"]
    p_wall = 0.5 * (d["fwall_y_lo"] - d["fwall_y_hi"]) / n / (s.Lx * s.Lz)
    db = b.flow_diag()
    rb = b.result()
    # kinetic part from the components the forcing does not stream (T_x also
    # holds the imposed profile's u^2)
    t_thermal = 0.5 * (rb["T"][1] + rb["T"][2])
    p_bulk = rho_b * t_thermal + db["virial"] / db["samples"] / (3.0 * b.Lx * b.Lz * b.h)
    assert p_wall == pytest.approx(p_bulk, rel=0.05), (p_wall, p_bulk)


@pytest.mark.slow
def test_isothermal_sound_speed_of_the_bulk_liquid():
    # c^2 = dp/drho at T = 1 from the virial pressure of the bulk periodic box
    # at densities 0.78 and 0.82 (the macro model's equation of state reading
    # compares its artificial c^2 = 200 with this); kinetic part from the
    # thermostatted temperature
    ps = []
    for rho in (0.78, 0.82):
        b, pb = _bulk(rho, 2000)
        b.run(2000 + 8000)
        d = b.flow_diag()
        r = b.result()
        rho_b = b.n_fluid / (b.Lx * b.Lz * b.h)
        ps.append((rho_b, rho_b * float(np.mean(r["T"])) + d["virial"] / d["samples"] / (3.0 * b.Lx * b.Lz * b.h)))
    c2 = (ps[1][1] - ps[0][1]) / (ps[1][0] - ps[0][0])
    print("bulk pressures", ps, "c2", c2)
    assert ps[0][1] < ps[1][1]
    assert 10.0 < c2 < 30.0
