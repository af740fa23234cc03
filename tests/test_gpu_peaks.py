"""The device-rate kernels behind the measured-peak roofline fractions: every
rate is positive and no rate exceeds the published dense peak of the MI355X
(a rate above it would mean the kernel did less work than it counts)."""
import pytest

from paper_1812_07607_amd import ops

pytestmark = pytest.mark.gpu

PUBLISHED = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0}  # TFLOP/s, dense
HBM_GBPS = 8000.0


def test_measured_peaks_are_plausible():
    pk = ops.measure_peaks()
    for fmt, peak in PUBLISHED.items():
        assert 0.2 * peak < pk[fmt] <= 1.05 * peak, (fmt, pk)
    assert 0.2 * HBM_GBPS < pk["hbm_copy_GBps"] <= 1.05 * HBM_GBPS, pk
    # the LDS-fed loop at two waves per SIMD cannot beat the published rate
    assert 0.2 * PUBLISHED["bf16"] < pk["bf16_lds_fed_candidate_loop"] <= 1.05 * PUBLISHED["bf16"], pk
