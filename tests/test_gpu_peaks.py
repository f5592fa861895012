"""The achievable-rate probe of the device (hmd_measure_peaks) through the
C ABI: every rate positive and below the published peaks it is reported
beside (FP32 157.3 TFLOP/s counting packed instructions, HBM 8 TB/s)."""
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
from paper_1603_04628_amd import binding as B  # noqa: E402


def test_measured_peaks_are_plausible():
    p = B.measure_peaks(hmd.Context())
    assert 1.0 < p["fp32_fma_tflops"] < 157.3
    assert 0.1 < p["fp32_rcp_tops"] < p["fp32_fma_tflops"]
    assert 1.0 <= p["rcp_cost_in_fma"] < 16.0
    assert 100.0 < p["copy_gbs"] < 8000.0
