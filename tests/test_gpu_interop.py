"""Device-pointer entry points (*_dev) against their host forms: the same
values land in torch tensors on the current stream."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
torch = pytest.importorskip("torch")
from paper_1603_04628_amd import binding as B  # noqa: E402


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(4, 20, n), rng.uniform(0.001, 0.05, n)])
    y = 0.004 * X[:, 0] ** 3 * X[:, 1] + rng.normal(0, 0.003, n)
    return X, y


def test_gp_predict_dev_equals_host():
    ctx = hmd.Context()
    X, y = _data(60, 1)
    g = B.GP(ctx, X, y, np.full(60, 0.003), B.gp_hyper(ranges=(16.0, 0.049)))
    Xq, _ = _data(77, 2)  # several query blocks and a ragged tail
    m_h, v_h = g.predict(Xq)
    m_d, v_d = g.predict_dev(torch.tensor(Xq, device="cuda"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m_d.cpu().numpy(), m_h)
    np.testing.assert_array_equal(v_d.cpu().numpy(), v_h)


def test_gp_predict_dev_prior():
    ctx = hmd.Context()
    g = B.GP(ctx, np.zeros((0, 2)), np.zeros(0), None, B.gp_hyper(ranges=(16.0, 0.049)))
    m_d, v_d = g.predict_dev(torch.tensor([[5.0, 0.01], [9.0, 0.02]], device="cuda"))
    m_h, v_h = g.predict(np.array([[5.0, 0.01], [9.0, 0.02]]))
    np.testing.assert_array_equal(m_d.cpu().numpy(), m_h)
    np.testing.assert_array_equal(v_d.cpu().numpy(), v_h)


def test_ens_predict_dev_equals_host():
    ctx = hmd.Context()
    X, y = _data(64, 3)
    e = B.Ensemble(ctx, X, y, B.ens_cfg(members=3, hidden=32, iters=50))
    Xq, _ = _data(301, 4)
    m_h, s_h = e.predict(Xq)
    m_d, s_d = e.predict_dev(torch.tensor(Xq, device="cuda"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m_d.cpu().numpy(), m_h)
    np.testing.assert_array_equal(s_d.cpu().numpy(), s_h)


def test_md_flux_batch_dev_equals_host():
    p = hmd.Params(Lx_nom=12.0, Lz_nom=12.0, n_equil=100)
    jobs = [(5.0, 0.02, 1, 200), (7.5, 0.01, 2, 200)]
    host = hmd.md_flux_batch(hmd.Context(p), jobs)
    f, se, st = hmd.md_flux_batch_dev(hmd.Context(p), jobs)
    # independent runs of the same seeds: same start, trajectories equal to
    # FP32 force rounding over 300 steps, so the fluxes agree closely
    np.testing.assert_allclose(f.cpu().numpy(), [r["flux"] for r in host], rtol=0.05, atol=0.02)
    assert st.cpu().tolist() == [r["status"] for r in host]
    assert np.all(se.cpu().numpy() > 0)
