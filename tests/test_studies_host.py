"""Host-side pieces of the Sec. 3 study runner (no GPU): the channel's
subdomains, the forcing tables and Eq. error."""
import numpy as np
import pytest

import studies


def test_subdomains_of_the_paper_channel():
    # Eqs. subsEq and heightEq with h_1 = 10, a = 2, L = 200: inlet 10, the
    # throat pair at s = 80, 120, and the paper's initial densities at N = 5
    h = studies.heights(5)
    assert h[0] == 10.0 and h[1] == pytest.approx(h[4], rel=1e-12) and h[2] == pytest.approx(h[3], rel=1e-12)
    assert h[2] == pytest.approx(10.0 + 2.0 * (np.cos(0.8 * np.pi) - 1.0), rel=1e-12)
    assert np.array_equal(studies.initial_rho(5), np.array(studies.RHO0))
    r10 = studies.initial_rho(10)
    assert np.array_equal(r10[::2], np.array(studies.RHO0))
    assert r10[9] == pytest.approx(0.5 * (studies.RHO0[4] + studies.RHO0[0]), rel=1e-12)  # across the ring's seam


def test_forcing_tables():
    f = studies.forcing_table("sine", 200, 100, 0.01)
    assert f[0] == 0.0 and f[25] == pytest.approx(0.01, rel=1e-12) and f[75] == pytest.approx(-0.01, rel=1e-12)
    r = studies.forcing_table("ramp", 200, 100, 0.01)
    assert r[25] == pytest.approx(0.01 * (1.0 + 0.25 * 25 / 200), rel=1e-12)
    c = studies.forcing_table("chirp", 200, 100, 0.01)
    # the instantaneous period grows from 10 to 100 steps: zero crossings
    # (half periods) are close together early and far apart late
    z = np.nonzero(np.diff(np.sign(c[1:])) != 0)[0]
    gaps = np.diff(z)
    assert gaps[0] <= 7 and gaps[-1] >= 35 and np.abs(c).max() <= 0.01
    with pytest.raises(ValueError):
        studies.forcing_table("square", 10, 5, 0.01)


def test_eq_error():
    Q = np.array([1.0, -2.0, 1.0])
    assert studies.eq_error(np.zeros(3), Q) == 100.0  # an empty database predicts zero flow
    assert studies.eq_error(Q, Q) == 0.0
    assert studies.eq_error([1.5, -2.0, 0.5], Q) == pytest.approx(25.0)
    assert np.allclose(studies.eq_error_series([1.5, -2.0, 0.5], Q), [50.0, 100.0 * 0.5 / 3.0, 25.0])
