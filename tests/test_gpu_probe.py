"""The ALU issue-rate probe the sweep kernels' roofline is priced against.
At the 2.4 GHz peak engine clock a compute unit issues at most one FP64 FMA
per lane per clock (64 lanes: the published 78.6 TFLOP/s FP64 vector peak)
and at most two 32-bit integer adds (gfx950 issues 32-bit VALU work at up to
twice the FP64 rate), so the mixed kind, half of each, is bounded by 4/3 of
one per lane per clock.  Each kind must reach a quarter of its bound, and bad
arguments are refused before any launch."""
import pytest

from paper_1902_08154_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_08154_amd.api import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind,per_clock", [(_lib.QP_PROBE_F64_FMA, 1.0), (_lib.QP_PROBE_I32_ADD, 2.0),
                                            (_lib.QP_PROBE_MIXED, 4.0 / 3.0)])
def test_probe_rate_within_the_clock_bound(ctx, kind, per_clock):
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    bound = n_cu * 64 * 2.4e9 * per_clock
    r = ctx.qp_alu_probe(kind, 1 << 12)
    print(f"kind {kind}: {r / 1e12:.2f} T lane-ops/s ({r / bound:.3f} of {bound / 1e12:.1f} T)", flush=True)
    assert 0.25 * bound < r <= 1.05 * bound


def test_probe_refuses_bad_arguments(ctx):
    from paper_1902_08154_amd.api import QPError
    for kind, iters in ((3, 16), (-1, 16), (0, 0), (0, (1 << 24) + 1)):
        with pytest.raises(QPError):
            ctx.qp_alu_probe(kind, iters)
