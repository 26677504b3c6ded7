"""Measurement support: the achievable-MFMA probe returns plausible rates
(positive, below twice the published dense peaks, BF16 above FP32)."""
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
