"""The allocation-free entry point md_series_stats_noalloc against the
entry point it varies, md_series_stats_dev, through the C ABI: two calls in
a row (the second smaller), the same kernels on a fixed device scratch, and
sizes beyond the scratch rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
from paper_1603_04628_amd import binding as B  # noqa: E402
from oracle import stats as ostats  # noqa: E402


def _rows(seed, S, n, phi):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((S, n))
    x = np.empty_like(e)
    x[:, 0] = e[:, 0]
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return 0.5 + 0.01 * x


def test_noalloc_equals_the_allocating_form():
    import torch
    ctx = hmd.Context(hmd.Params(Lx_nom=12.0, Lz_nom=12.0))
    for S, n, phi in ((16, 40000, 0.99), (3, 1001, 0.7)):  # the second call smaller
        xs = _rows(S * 7 + n, S, n, phi)
        x = torch.from_numpy(xs).cuda()
        out = torch.zeros((S, 4), dtype=torch.float64, device="cuda")
        B.series_stats_noalloc(ctx, x, out)
        ref = B.series_stats_dev(ctx, x)
        torch.cuda.synchronize()
        a, r = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, r), np.abs(a - r).max()
        for k in range(S):
            m, se = ostats.geyer(xs[k])
            assert a[k, 0] == pytest.approx(m, rel=1e-12)
            assert a[k, 1] == pytest.approx(se, rel=1e-10)
        # the block rule needs no scratch
        outb = torch.zeros((S, 4), dtype=torch.float64, device="cuda")
        B.series_stats_noalloc(ctx, x, outb, n_blocks=20)
        refb = B.series_stats_dev(ctx, x, n_blocks=20)
        torch.cuda.synchronize()
        assert np.array_equal(outb.cpu().numpy(), refb.cpu().numpy())


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    ctx = hmd.Context(hmd.Params(Lx_nom=12.0, Lz_nom=12.0))
    x = torch.zeros((65, 1 << 15), dtype=torch.float64, device="cuda")  # 65 * 32768 > 2^21
    out = torch.zeros((65, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(hmd.HmdError, match="fixed scratch"):
        B.series_stats_noalloc(ctx, x, out)
