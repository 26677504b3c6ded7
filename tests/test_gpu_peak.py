"""Measurement support: the achievable-MFMA probe returns plausible rates
(positive, below twice the published dense peaks, BF16 above FP32) and a
plausible shader clock (the MI355X tops out at 2.4 GHz), consistent with the
rate: the FP32 rate cannot exceed 256 CUs x 256 flop per cycle at that clock."""
import pytest

pytestmark = pytest.mark.gpu


def test_peak_mfma_rates_are_plausible():
    import paper_1705_07112_amd as cpa
    f32 = cpa.peak_mfma("fp32", iters=2000)
    bf16 = cpa.peak_mfma("bf16", iters=2000)
    print(f"achievable MFMA: fp32 {f32:.1f} TFLOP/s, bf16 {bf16:.1f} TFLOP/s", flush=True)
    assert 10.0 < f32 < 2 * 157.3
    assert f32 < bf16 < 2 * 2516.6
    with pytest.raises(cpa.CpaError):
        cpa.peak_mfma("fp32", iters=0)


def test_peak_mfma_clock_is_plausible():
    import paper_1705_07112_amd as cpa
    f32, ghz = cpa.peak_mfma("fp32", iters=4000, clock=True)
    print(f"fp32 {f32:.1f} TFLOP/s at {ghz:.3f} GHz; rate / (256 CU x 256 flop x clock) = "
          f"{f32 / (256 * 256 * ghz * 1e-3):.3f}", flush=True)
    assert 0.5 < ghz < 2.6
    assert f32 <= 256 * 256 * ghz * 1e-3 * 1.02
