"""fsmmc_measure_ceilings through the C ABI: the measured unit rates are
positive and below 1.2x the spec-sheet peaks (a rate above the spec would
mean the kernels' work is counted wrong), and bad sizes are rejected."""
import pytest

pytestmark = pytest.mark.gpu


def test_ceilings_plausible():
    from paper_2503_17405_amd import fsmmc as F
    c = F.measure_ceilings(0, 256 << 20)
    spec = dict(hbm_copy_gbps=8000.0, mfma_bf16_tflops=2500.0, mfma_f32_tflops=157.3, valu_f32_tflops=78.6,
                valu_f64_tflops=78.6)
    for k, peak in spec.items():
        assert 0.0 < c[k] < 1.2 * peak, (k, c[k])
    # the hardware exp2 runs no faster than an FMA per lane
    assert 0.0 < c["exp_f32_gops"] * 1e9 < 1.2 * c["valu_f32_tflops"] * 1e12 / 2
    assert c["cus"] > 0 and c["clock_mhz"] > 0


def test_ceilings_argument_errors():
    from paper_2503_17405_amd import fsmmc as F
    for size in (1 << 20, (64 << 20) + 8):
        with pytest.raises(F.FsmmcError) as e:
            F.measure_ceilings(0, size)
        assert e.value.status == F.EINVAL
