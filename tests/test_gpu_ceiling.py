"""The MFMA ceiling measurement behind the roofline context: a kernel of
independent MFMAs of one kind reaches at most the published dense peak, and
its rate agrees with that peak scaled by the shader clock it measured (the
matrix cores run at full rate; a sustained load lowers the clock)."""
import pytest

pytestmark = pytest.mark.gpu

PEAK = {"fp8": 5000.0, "bf16": 2500.0, "fp32": 157.3}   # TFLOP/s at 2.4 GHz


@pytest.mark.parametrize("kind", ["fp32", "bf16", "fp8"])
def test_mfma_ceiling_is_the_clock_scaled_peak(gpu_lib, kind):
    print("mfma ceiling, %s" % kind, flush=True)
    c = gpu_lib.mfma_ceiling(kind)
    print(c, flush=True)
    assert 0.0 < c["tflops"] <= PEAK[kind] * 1.001
    assert 0.5 < c["clock_ghz"] < 2.6
    scaled = PEAK[kind] * c["clock_ghz"] / 2.4
    assert 0.85 * scaled <= c["tflops"] <= 1.05 * scaled
