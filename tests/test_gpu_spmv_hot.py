"""GPU parity of the hot-column layout (wc_spmv_prepare, wc_spmv_hot): the
prepared column ids and hot ids equal their plain definition computed on the
host, and every product is bit-identical to wc_spmv on the original matrix with
the same mode and tune (same kernels and summation order) and within the
oracle's 1e-5 bound, in every mode and at the scale-22 size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_to_dev, say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def expected_layout(g, hot):
    """Columns ranked by entry count (most first, ties by id): the hot ones map
    to their rank, the others to hot + id."""
    cnt = np.bincount(g.col, minlength=g.n)
    order = np.lexsort((np.arange(g.n), -cnt))
    rank = np.full(g.n, -1, np.int64)
    rank[order[:hot]] = np.arange(hot)
    col_hot = np.where(rank[g.col] >= 0, rank[g.col], hot + g.col.astype(np.int64))
    return col_hot.astype(np.int32), order[:hot].astype(np.int32)


def both(ctx, g, val, x, hot, mode, tune=None):
    da = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dv, dx = f32_to_dev(val), f32_to_dev(x)
    a_hot, ids = ctx.spmv_prepare(da, hot)
    say(f"spmv_hot n={g.n} m={g.m} hot={hot} mode={mode} tune={tune.as_dict() if tune else None}")
    y = ctx.spmv_hot(a_hot, ids, dv, dx, mode=mode, tune=tune)
    y0 = ctx.spmv(da, dv, dx, mode=mode, tune=tune)
    torch.cuda.synchronize()
    return a_hot, ids, y.cpu().numpy(), y0.cpu().numpy()


@pytest.fixture(scope="module")
def c1(c1_graph):
    g, _ = c1_graph
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    return g, val, x, y_ref, b


@pytest.mark.parametrize("mode", MODES)
def test_layout_and_products_scale12(ctx, c1, mode):
    g, val, x, y_ref, b = c1
    for hot in (0, 1, 100, 2000, g.n):
        a_hot, ids, y, y0 = both(ctx, g, val, x, hot, mode)
        col_hot, hot_ids = expected_layout(g, hot)
        assert np.array_equal(a_hot.col.cpu().numpy(), col_hot), hot
        assert np.array_equal(ids.cpu().numpy(), hot_ids), hot
        assert np.array_equal(y.view(np.uint32), y0.view(np.uint32)), hot
        assert oracle.spmv_check(y_ref, b, y) == (0, -1), hot


@pytest.mark.parametrize("tune", [dict(block_threads=64), dict(block_threads=128, items_per_lane=1),
                                  dict(block_threads=1024, items_per_lane=16), dict(threshold=1, grid_blocks=3)])
def test_grid_tunes_bit_identical(ctx, c1, tune):
    g, val, x, y_ref, b = c1
    _, _, y, y0 = both(ctx, g, val, x, 3000, "grid", wc.make_tune(**tune))
    assert np.array_equal(y.view(np.uint32), y0.view(np.uint32))
    assert oracle.spmv_check(y_ref, b, y) == (0, -1)


def test_edge_cases_and_refusals(ctx):
    n = 1500
    for name, edges in (("empty_rows", [(7, 3), (7, 9), (1000, 1)]), ("no_entries", []),
                        ("one_huge_row", [(3, j % n) for j in range(50000)])):
        g = synth.graph_from_edges(n, edges)[0]
        val, x = synth.values(g.m, seed=31), synth.vector_x(g.n, seed=37)
        y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
        for mode in MODES:
            _, _, y, y0 = both(ctx, g, val, x, min(64, n), mode)
            assert np.array_equal(y.view(np.uint32), y0.view(np.uint32)), (name, mode)
            assert oracle.spmv_check(y_ref, b, y) == (0, -1), (name, mode)
    g = synth.graph_from_edges(10, [(0, 1)])[0]
    da = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    for hot in (-1, 11):
        with pytest.raises(wc.WcError) as ei:
            ctx.spmv_prepare(da, hot)
        assert ei.value.status == -1
    torch.cuda.synchronize()


def test_scale22_bit_identical_and_within_bound(ctx):
    say("generating scale-22 matrix for the hot-column layout")
    g = synth.rmat_csr(22, 1 << 26)
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    for mode in ("grid", "block"):
        _, _, y, y0 = both(ctx, g, val, x, 65536, mode)
        assert np.array_equal(y.view(np.uint32), y0.view(np.uint32)), mode
        assert oracle.spmv_check(y_ref, b, y) == (0, -1), mode
