"""The issue-rate probes behind the roofline (lens_peak_rate): the rates the
credited work is priced at.  The vector ALU's full-rate kinds run near the
nominal 256 CU x 4 SIMD x 16 lanes x 2.4 GHz; an FP32 transcendental costs the
bench's TRANS_SLOTS full-rate slots (CDNA4 issues them at half rate) and does
not issue beside the FMAs; the FP16 and BF16 products reach the dense
matrix-core peak."""
import pytest

from gpu_cases import say

pytestmark = pytest.mark.gpu

FULL_RATE = ["fma_f64", "mul_f64", "add_f64", "cvt_f64_f32", "ldexp_f64", "frexp_mant_f64", "rndne_f64"]
TRANS = ["exp_f32", "log_f32", "rsq_f32", "rcp_f32"]


@pytest.fixture(scope="module")
def rates():
    from paper_2503_08586_amd import binding
    say("case: instruction issue-rate probes")
    with binding.LensContext(0) as ctx:
        r = {name: ctx.peak_rate(name) for name in binding.PEAK_OPS}
    for k, v in r.items():
        say("%s: %.4g" % (k, v))
    return r


def test_full_rate_vector_ops(rates):
    import bench
    for name in FULL_RATE:
        assert 0.8 <= rates[name] / bench.PEAK_SLOT_PER_S <= 1.0, name
    # not packed: at most the two-lanes-per-slot rate
    assert 0.8 <= rates["fma_f32"] / bench.PEAK_SLOT_PER_S <= 2.0


def test_transcendental_slot_cost(rates):
    import bench
    for name in TRANS:
        slots = rates["fma_f64"] / rates[name]
        assert abs(slots - bench.TRANS_SLOTS) <= 0.4, (name, slots)
    # alternating with FMAs, a transcendental still takes its slots: the mix
    # runs at the harmonic combination of the two rates (within 10%)
    both = 2.0 / (1.0 / rates["fma_f64"] + 1.0 / rates["exp_f32"])
    assert abs(rates["fma_f64_exp_f32"] / both - 1.0) <= 0.1


def test_matrix_core_products(rates):
    import bench
    for name in ("mfma_f16", "mfma_bf16"):
        assert 0.9 <= rates[name] / bench.PEAK_BF16_FLOP_S <= 1.02, name
    assert 0 < rates["mfma_f16_fma_f64"] <= 1.05 * rates["fma_f64"]


def test_unknown_instruction_kind():
    from paper_2503_08586_amd import binding
    with binding.LensContext(0) as ctx:
        for op in (-1, len(binding.PEAK_OPS)):
            with pytest.raises(binding.LensError):
                binding.lens_peak_rate(ctx.ctx, op)
