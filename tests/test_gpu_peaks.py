"""The device-rate probe (include/npm_probe.h) on the MI355X: every figure is
positive and below the published peak it is measured against (FP32 matrix
157.3 TFLOP/s, BF16 matrix 2,500 TFLOP/s, HBM 8,000 GB/s; the copy counts
bytes read plus written, so it too stays under the HBM peak), and high
enough that the probe is not broken (a tenth of the peak at least)."""
import pytest

from paper_2504_04315_amd import npm as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def test_measured_peaks_are_plausible(torch):
    p = B.measure_peaks(reps=2)
    print({k: round(v, 1) for k, v in p.items()})
    for key, peak in (("mfma_f32_tflops", 157.3), ("mfma_bf16_tflops", 2500.0),
                      ("hbm_read_gbs", 8000.0), ("hbm_copy_gbs", 8000.0)):
        assert 0.1 * peak < p[key] < 1.02 * peak, (key, p[key])
