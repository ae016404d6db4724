"""The device's sustained FMA rate (akra_fma_rate), the ceiling printed beside the roofline peaks."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,peak", [("fp64", 78.6), ("fp32", 157.3)])
def test_fma_rate_is_positive_and_below_the_published_peak(prec, peak):
    from paper_2606_06175_amd.akra import fma_rate
    r = fma_rate(prec)
    print("%s sustained FMA rate %.1f TFLOP/s" % (prec, r), flush=True)
    # plain (not packed) FMAs: FP32 retires at the FP64 rate, below 78.6 TFLOP/s either way
    assert 10.0 < r < 1.02 * min(peak, 78.6)


@pytest.mark.parametrize("chains,valu,waves", [(4, 0, 2), (2, 4, 1)])
def test_mfma_rate_is_positive_and_below_the_published_peak(chains, valu, waves):
    from paper_2606_06175_amd.akra import mfma_rate
    r = mfma_rate(chains, valu, waves)
    print("v_mfma_f32_32x32x2_f32, %d chains, %d FMA pairs between products, %d waves per SIMD: %.1f TFLOP/s"
          % (chains, valu, waves, r), flush=True)
    assert 5.0 < r < 1.02 * 157.3
