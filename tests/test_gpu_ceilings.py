"""Measured ceilings of the GPU (ccd_measure_ceilings): plausible and below
the published peaks (HBM 8 TB/s; FP64 78.6, FP32 157.3, BF16 about 2500
TFLOP/s dense), and the FP64 rates above what the ladder kernel reaches."""
import pytest

pytestmark = pytest.mark.gpu

ccd = pytest.importorskip("paper_1611_06765_amd.ccd")


def test_ceilings_are_plausible():
    import torch
    assert torch.cuda.is_available()
    c = ccd.measure_ceilings(1 << 28)
    assert 1000.0 < c["hbm_copy_gbs"] < 8000.0
    for k, peak in (("fp64_mfma_16x16x4_tflops", 78.6), ("fp64_mfma_4x4x4_tflops", 78.6),
                    ("fp32_mfma_16x16x4_tflops", 157.3), ("bf16_mfma_16x16x32_tflops", 2600.0)):
        assert 0.1 * peak < c[k] <= 1.02 * peak, (k, c[k])
