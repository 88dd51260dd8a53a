"""The register-only VALU probes (pa_probe_valu, pa_probe_goldilocks): they
run, report positive rates, and order as their instruction counts say (8
VALU instructions per 30-bit butterfly, 2 per plain pair, 42 per butterfly
modulo 2^64 - 2^32 + 1 with a general twiddle, about 24 with a shift
twiddle)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2105_13678_amd as pa
    pa.lib()
    return pa


def test_probes_report_ordered_rates(pa):
    bfly, plain = pa.probe_valu(0)
    gl_mul, gl_shift = pa.probe_goldilocks(0)
    print(f"[case] probes: 30-bit {bfly:.3g}/s, plain {plain:.3g}/s, mod P {gl_mul:.3g}/s and {gl_shift:.3g}/s", flush=True)
    assert 0 < gl_mul < gl_shift < bfly < plain
    # the counted peak of the 30-bit butterfly (256 CUs x 64 lanes x 2.4 GHz / 8) within a factor 2
    assert 0.5 * 4.9152e12 < bfly < 2 * 4.9152e12
