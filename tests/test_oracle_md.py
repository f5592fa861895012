"""Pins for the FP64 MD oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, symmetry, exact invariants, brute force,
or textbook properties of velocity Verlet.  CPU only.
"""
import os

import numpy as np
import pytest

from oracle import md

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# the literal 12 x 12 box of the small channel (774 fluid atoms at h = 6)
SMALL = dict(Lx_nom=12.0, Lz_nom=12.0)


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- generator
def test_philox_known_answers():
    for row in _golden("philox4x32_10_kat.txt"):
        vals = [int(t, 16) for t in row]
        out = md.philox4x32_10(vals[0:4], vals[4:6])
        assert list(out) == vals[6:10]


# ---------------------------------------------------------------- potential
def test_lj_closed_forms():
    for r, u, f in _golden("lj_closed_form.txt"):
        r, u, f = float(r), float(u), float(f)
        assert md.lj_energy(r) == pytest.approx(u, abs=1e-14)
        assert md.lj_force(r) == pytest.approx(f, abs=1e-13)


def test_lj_wall_parameters_scale():
    # U(r; eps, sig) = eps U(r/sig; 1, 1): the wall-fluid pair uses the same law
    assert md.lj_energy(1.5, 0.2, 0.75) == pytest.approx(0.2 * md.lj_energy(2.0), rel=1e-14)


def _two_atoms(positions, **kw):
    p = md.Params(wall_layers=0, n_fluid=2, **SMALL, **kw)
    s = md.System(6.0, 0.0, 0, p)
    x = np.array(positions, dtype=float)
    s.set_state(x, np.zeros((2, 3)))
    return s


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_pair_force_sign_and_value(axis):
    # r = 1: U = 0, |F| = 24, repulsive: atom 0 is pushed away from atom 1
    a = np.array([5.0, 3.0, 5.0])
    b = a.copy()
    b[axis] += 1.0
    s = _two_atoms([a, b])
    f, pe = s.forces_brute()
    exp = np.zeros(3)
    exp[axis] = -24.0
    np.testing.assert_allclose(f[0], exp, atol=1e-12)
    np.testing.assert_allclose(f[1], -exp, atol=1e-12)
    # shifted energy: U(1) - U(r_c) = 0 + 0.016316891136
    assert pe == pytest.approx(0.016316891136, abs=1e-12)


def test_pair_force_through_periodic_boundary():
    s = _two_atoms([[0.3, 3.0, 4.0], [0.0, 3.0, 4.0]])
    L = s.Lx
    s = _two_atoms([[0.3, 3.0, 4.0], [L - 0.7, 3.0, 4.0]])
    f, _ = s.forces_brute()
    np.testing.assert_allclose(f[0], [24.0, 0, 0], atol=1e-11)
    fc, _ = s.forces_cells()
    np.testing.assert_allclose(fc, f, atol=1e-12)


def test_pair_cutoff_is_strict():
    s = _two_atoms([[5.0, 3.0, 5.0], [7.5, 3.0, 5.0]])
    f, pe = s.forces_brute()
    assert np.all(f == 0.0) and pe == 0.0
    s = _two_atoms([[5.0, 3.0, 5.0], [7.49, 3.0, 5.0]])
    f, _ = s.forces_brute()
    assert f[0, 0] > 0.0  # attractive tail pulls atom 0 toward +x


# ---------------------------------------------------------------- geometry
def test_wall_lattice_geometry():
    s = md.System(6.0, 0.0, 0, md.Params(**SMALL))
    xw = s.wall()
    n = int(round(s.Lx / (4.0 ** (1.0 / 3.0))))
    assert s.n_wall == 2 * 4 * 2 * n * n
    ys = np.unique(np.round(xw[:, 1], 12))
    # innermost planes at 0 and h: h is the gap between them
    assert ys.min() == pytest.approx(-3 * 0.5 * 4 ** (1 / 3)) and 0.0 in ys and 6.0 in ys
    # FCC at number density 1: nearest neighbours at a/sqrt(2) = 2^(1/6)
    layer = xw[np.abs(xw[:, 1]) < 1e-12]
    d = layer[:, None, [0, 2]] - layer[None, :, [0, 2]]
    d = d - s.Lx * np.round(d / s.Lx)
    r = np.sqrt((d ** 2).sum(-1))
    r = r[r > 1e-9]
    assert r.min() == pytest.approx(2 ** (1 / 6), rel=1e-12)
    # 4 layers of 2 n^2 atoms in a cube of side a/2 stacked: density 1
    assert len(layer) / (s.Lx * s.Lz) * 2 / (4 ** (1 / 3)) == pytest.approx(1.0, rel=1e-12)


def test_atom_at_mid_gap_feels_no_net_wall_force():
    p = md.Params(n_fluid=1, **SMALL)
    s = md.System(6.0, 0.0, 0, p)
    a = 4 ** (1 / 3)
    # above a hollow site of the (100) face: in-plane forces cancel by symmetry
    x = np.array([[2 * a + 0.5 * a, 0.6, 2 * a]])
    s.set_state(x, np.zeros((1, 3)))
    f, _ = s.forces_brute()
    assert abs(f[0, 0]) < 1e-12 and abs(f[0, 2]) < 1e-12
    assert f[0, 1] > 0  # pushed away from the lower wall
    # at mid-gap the two walls are mirror images: no net normal force
    x = np.array([[2 * a + 0.5 * a, 3.0, 2 * a]])
    s.set_state(x, np.zeros((1, 3)))
    f, _ = s.forces_brute()
    assert np.all(np.abs(f[0]) < 1e-12)


# ---------------------------------------------------------------- start
def test_initial_state():
    p = md.Params(**SMALL)
    s = md.System(6.0, 0.02, 3, p)
    x, v = s.get_state()
    assert s.n_fluid == round(0.8 * s.Lx * s.Lz * 6.0)
    assert np.abs(v.mean(0)).max() < 1e-14
    assert (v ** 2).sum() / (3 * s.n_fluid) == pytest.approx(1.0, abs=1e-13)
    assert x[:, 1].min() >= 1.0 - 1e-12 and x[:, 1].max() <= 5.0 + 1e-12
    from scipy.spatial.distance import pdist
    d = x[:, None, :] - x[None, :, :]
    d[..., 0] -= s.Lx * np.round(d[..., 0] / s.Lx)
    d[..., 2] -= s.Lz * np.round(d[..., 2] / s.Lz)
    r = np.sqrt((d ** 2).sum(-1))[np.triu_indices(s.n_fluid, 1)]
    assert r.min() > 0.95
    # Box-Muller draws: roughly normal, unit variance per component before rescale
    assert abs(np.mean(v ** 4) / np.mean(v ** 2) ** 2 - 3.0) < 0.5
    x2, v2 = md.System(6.0, 0.02, 3, p).get_state()
    assert np.array_equal(x, x2) and np.array_equal(v, v2)
    x3, v3 = md.System(6.0, 0.02, 4, p).get_state()
    assert not np.array_equal(v, v3)
    del pdist


# ---------------------------------------------------------------- forces
@pytest.fixture(scope="module")
def small_equilibrated():
    p = md.Params(**SMALL)
    s = md.System(6.0, 0.02, 1, p)
    s.run(1000)
    return s


def test_brute_force_equals_cell_list(small_equilibrated):
    s = small_equilibrated
    fb, peb = s.forces_brute()
    fc, pec = s.forces_cells()
    assert np.abs(fb - fc).max() <= 1e-13 * np.abs(fb).max()
    assert pec == pytest.approx(peb, rel=1e-13)


def test_newton_third_law_without_walls():
    p = md.Params(wall_layers=0, **SMALL)
    s = md.System(6.0, 0.0, 2, p)
    x, v = s.get_state()
    rng = np.random.default_rng(0)
    s.set_state(x + rng.uniform(-0.05, 0.05, x.shape) * [1, 0, 1], v)
    f, _ = s.forces_brute()
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).sum()


def test_cell_lists_partition(small_equilibrated):
    s = small_equilibrated
    cell_of, counts, order = s.cells()
    x, _ = s.get_state()
    nx, ny, nz = s.ncell
    assert counts.sum() == s.n_fluid
    assert sorted(order.tolist()) == list(range(s.n_fluid))
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for c in range(nx * ny * nz):
        members = order[start[c]:start[c] + counts[c]]
        assert np.all(np.diff(members) > 0)  # stable: ascending atom id
        assert np.all(cell_of[members] == c)
    cx, cy, cz = cell_of % nx, (cell_of // nx) % ny, cell_of // (nx * ny)
    wx, wy, wz = s.Lx / nx, 6.0 / ny, s.Lz / nz
    for c_a, x_a, w_a in ((cx, x[:, 0], wx), (cy, x[:, 1], wy), (cz, x[:, 2], wz)):
        assert np.all(x_a >= c_a * w_a - 1e-12) and np.all(x_a < (c_a + 1) * w_a + 1e-12)


# ---------------------------------------------------------------- integrator
def test_nve_energy_error_scales_as_dt_squared(small_equilibrated):
    x0, v0 = small_equilibrated.get_state()
    sd = {}
    for dt in (0.004, 0.002):
        s = md.System(6.0, 0.0, 1, md.Params(dt=dt, **SMALL))
        s.set_state(x0, v0)
        tr = s.run(int(round(2.0 / dt)), thermostat=False, energy=True)
        sd[dt] = tr.std()
        assert abs(tr[-1] - tr[0]) < 5e-4  # no secular drift over 2 tau
    assert 3.0 < sd[0.004] / sd[0.002] < 5.0


def test_velocity_verlet_is_time_reversible(small_equilibrated):
    x0, v0 = small_equilibrated.get_state()
    s = md.System(6.0, 0.0, 1, md.Params(**SMALL))
    s.set_state(x0, v0)
    s.run(200, thermostat=False)
    x1, v1 = s.get_state()
    s.set_state(x1, -v1)
    s.run(200, thermostat=False)
    x2, v2 = s.get_state()
    d = x2 - x0
    d[:, 0] -= s.Lx * np.round(d[:, 0] / s.Lx)
    d[:, 2] -= s.Lz * np.round(d[:, 2] / s.Lz)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-8


# ---------------------------------------------------------------- thermostat / flux
def test_berendsen_holds_target_and_equipartition(small_equilibrated):
    x0, v0 = small_equilibrated.get_state()
    s = md.System(6.0, 0.0, 1, md.Params(n_equil=500, **SMALL))
    s.set_state(x0, v0)
    s.run(3500)
    r = s.result()
    Tx, Ty, Tz = r["T"]
    assert Ty == pytest.approx(1.0, abs=0.01)
    assert Tx == pytest.approx(1.0, abs=0.03) and Tz == pytest.approx(1.0, abs=0.03)


@pytest.mark.slow
def test_flux_symmetry_and_linear_response():
    # rho = 0.6 over the wall-plane gap keeps the 6-sigma channel liquid (at 0.8
    # the first layers reach a local density near freezing and the flow is tiny)
    p = md.Params(n_equil=3000, rho=0.6, **SMALL)
    res = {g: md.md_flux(6.0, g, 7, 8000, p) for g in (0.0, 0.1, -0.1, 0.2)}
    for g, r in res.items():
        assert r["status"] == 0, (g, r)
    z = res[0.0]
    assert abs(z["flux"]) <= 4 * z["flux_se"]
    a, b, c = res[0.1], res[-0.1], res[0.2]
    assert a["flux"] > 4 * a["flux_se"] and b["flux"] < -4 * b["flux_se"]
    # mirror symmetry x -> -x: q(-g) = -q(g) within the sampling error
    assert abs(a["flux"] + b["flux"]) <= 4 * np.hypot(a["flux_se"], b["flux_se"])
    # linear response: doubling the force doubles the flux
    assert 1.4 < c["flux"] / (0.5 * (a["flux"] - b["flux"])) < 2.6


# ---------------------------------------------------------------- statistics
def test_block_standard_error():
    n, nb = 20000, 20
    mean, se, m1, m2, B = md.block_stats(np.full(n, 2.5), nb)
    assert (mean, se, B) == (2.5, 0.0, 1000)
    # remainder dropped from the front
    s = np.concatenate([np.full(7, 1e9), np.ones(n)])
    assert md.block_stats(s, nb)[0] == 1.0
    # a linear ramp: block means are B (b + 1/2) - 1/2, b = 0..19; their sample
    # variance is B^2 * 35, so SE = B sqrt(35 / 20)
    mean, se, m1, m2, B = md.block_stats(np.arange(n, dtype=float), nb)
    assert mean == pytest.approx((n - 1) / 2)
    assert se == pytest.approx(B * np.sqrt(35.0 / 20.0), rel=1e-12)
    assert m2 - m1 == pytest.approx(10 * B)
    # white noise: SE ~ sigma / sqrt(n) (20 blocks -> ~16% scatter of the estimate)
    rng = np.random.default_rng(5)
    ses = [md.block_stats(rng.normal(0, 3.0, n), nb)[1] for _ in range(20)]
    assert np.mean(ses) == pytest.approx(3.0 / np.sqrt(n), rel=0.1)


def test_overlapping_atoms_are_reported_unstable():
    p = md.Params(n_equil=0, n_blocks=2, **SMALL)
    s = md.System(6.0, 0.0, 0, p)
    x, v = s.get_state()
    x[1] = x[0] + [0.05, 0.0, 0.0]
    s.set_state(x, v)
    s.run(4)
    assert s.result()["status"] == -4


def test_neighbor_sets_symmetric_and_nested(small_equilibrated):
    s = small_equilibrated
    nb = s.neighbors(2.8)
    nf = s.n_fluid
    pairs = {(i, int(j)) for i in range(nf) for j in nb[i] if j < nf}
    assert all((j, i) in pairs for i, j in pairs)
    inner = s.neighbors(2.5)
    assert all(set(inner[i].tolist()) <= set(nb[i].tolist()) for i in range(nf))
    # every in-cutoff neighbour contributes to the force: the pair count matches
    # the brute-force energy's pair count implied by a cut-off just above 0
    assert sum(len(a) for a in inner) < sum(len(a) for a in nb)


@pytest.mark.slow
def test_wide_channel_core_is_poiseuille():
    # h = 20 sigma, body force g: away from the wall layers the streaming
    # velocity follows the continuum solution u(y) = (rho g / 2 eta) y (h' - y)
    # up to an offset: a parabola, symmetric about the mid-plane, whose
    # curvature gives a shear viscosity in the range of the LJ liquid near
    # rho = 0.8, T = 1 (about 2 in reduced units)
    p = md.Params(Lx_nom=12.0, Lz_nom=12.0, n_equil=12000, thermo_axis=2)
    g = 0.02
    s = md.System(20.0, g, 3, p)
    s.run(24000)
    mvx, cnt = s.profile()
    y = (np.arange(len(mvx)) + 0.5) * p.bin_dy
    u = mvx / np.maximum(cnt, 1.0)
    core = (y > 4.0) & (y < 16.0)
    rho_core = cnt[core].sum() / cnt.sum() * s.n_fluid / (s.Lx * s.Lz * core.sum() * p.bin_dy)
    A = np.column_stack([np.ones(core.sum()), y[core], y[core] ** 2])
    c, *_ = np.linalg.lstsq(A, u[core], rcond=None)
    fit = A @ c
    r2 = 1.0 - np.sum((u[core] - fit) ** 2) / np.sum((u[core] - u[core].mean()) ** 2)
    assert r2 >= 0.9
    assert c[2] < 0.0
    assert abs(-c[1] / (2.0 * c[2]) - 10.0) < 1.0  # vertex at the mid-plane
    eta = -rho_core * g / (2.0 * c[2])
    assert 1.5 < eta < 3.0
    # the profile integrates to the measured mass flow rate per unit span
    r = s.result()
    q_profile = np.sum(mvx) / (s.Lx * s.Lz) / (24000 - 12000)
    assert q_profile == pytest.approx(r["flux"], rel=0.02)
