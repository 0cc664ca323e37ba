"""wc_spmv_noalloc (the entry point for callers that cannot allocate) against
wc_spmv with the same mode and tune: bit-identical y, and every row within the
oracle's bound |y - y_ref| <= 1e-5 * sum|a_ij x_j|.  Two calls in a row share
the fixed scratch array, the second on a smaller matrix."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_to_dev, say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu


def problem(scale, m):
    g = synth.rmat_csr(scale, m)
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    return g, val, x, y_ref, b


@pytest.fixture(scope="module")
def problems():
    return {16: problem(16, 1 << 20), 12: problem(12, 1 << 16)}


def both(ctx, g, val, x, mode, tune=None, stream=None):
    da = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dv, dx = f32_to_dev(val), f32_to_dev(x)
    out = torch.full((g.n,), float("nan"), dtype=torch.float32, device="cuda")
    say(f"spmv_noalloc n={g.n} m={g.m} mode={mode} tune={tune.as_dict() if tune else None}")
    wc.spmv_noalloc(da, dv, dx, out, mode=mode, tune=tune, stream=stream)
    ref = ctx.spmv(da, dv, dx, mode=mode, tune=tune, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("mode", ["grid", "block", "wave", "flat"])
def test_two_calls_second_smaller(ctx, problems, mode):
    for scale in (16, 12):
        g, val, x, y_ref, b = problems[scale]
        y, y_ctx = both(ctx, g, val, x, mode)
        assert np.array_equal(y.view(np.uint32), y_ctx.view(np.uint32)), (scale, mode)
        assert oracle.spmv_check(y_ref, b, y) == (0, -1), (scale, mode)


def test_tuned_and_on_a_side_stream(ctx, problems):
    g, val, x, y_ref, b = problems[12]
    side = torch.cuda.Stream()
    for tune in (wc.make_tune(threshold=2, items_per_lane=1, block_threads=128),
                 wc.make_tune(items_per_lane=16, block_threads=1024, grid_blocks=3)):
        with torch.cuda.stream(side):
            y, y_ctx = both(ctx, g, val, x, "grid", tune=tune, stream=side)
        assert np.array_equal(y.view(np.uint32), y_ctx.view(np.uint32))
        assert oracle.spmv_check(y_ref, b, y) == (0, -1)
