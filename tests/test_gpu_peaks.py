"""The peak-rate probes behind the roofline fractions: every measured rate is
positive and below the MI355X datasheet figure for the same unit, so no
probe's work was optimised away and none is mis-scaled."""
import pytest

pytestmark = pytest.mark.gpu

# MI355X datasheet: 8 TB/s HBM, 2.5 PFLOP/s dense BF16, 157.3 TFLOP/s FP32 vector.
# Generous upper bounds for the rest (256 CUs, 2.4 GHz): 256 LDS bytes, 64 LDS
# atomics and 256 transcendental lane-operations per clock per CU.
BOUNDS = {
    "hbm_bytes_per_s": 8.0e12,
    "lds_bytes_per_s": 256 * 2.4e9 * 256,
    "lds_atomics_per_s": 256 * 2.4e9 * 64,
    "fp32_fma_flop_per_s": 157.3e12,
    "sin_per_s": 256 * 4 * 64 * 2.4e9,
    "bf16_mfma_flop_per_s": 2.5e15,
    "lds_gather8_per_s": 256 * 2.4e9 * 32,        # 8-byte lane reads: at most 256 bytes per clock per CU
    "fp32_mfma_flop_per_s": 157.3e12,
}


def test_measured_peaks_are_physical():
    from paper_2009_00735_amd import native as nat
    ctx = nat.Context(0)
    p = nat.ar_measure_peaks(ctx)
    print(p)
    for k, hi in BOUNDS.items():
        assert 0.0 < p[k] <= 1.05 * hi, (k, p[k], hi)
    assert 0.2 < p["sin_beside_fma_time_ratio"] <= 1.2
    # random reads cannot beat conflict-free 16-byte reads per byte
    assert 8 * p["lds_gather8_per_s"] <= 1.05 * p["lds_bytes_per_s"]
