"""GPU parity of wc_spmv against the binary64 oracle: every row within
|y - y_ref| <= 1e-5 * sum|a_ij x_j|, bitwise reproducible per (mode, tune), and
the consolidation bookkeeping (buffered rows, dispatches) equal to the oracle's
count for the same threshold and scope."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_to_dev, say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def run(ctx, g, val, x, mode, stats=False, **tune):
    da = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    t = wc.make_tune(**tune) if tune else None
    say(f"spmv n={g.n} m={g.m} mode={mode} tune={tune}")
    res = ctx.spmv(da, f32_to_dev(val), f32_to_dev(x), mode=mode, tune=t, stats=stats)
    torch.cuda.synchronize()
    if stats:
        return res[0].cpu().numpy(), res[1]
    return res.cpu().numpy()


@pytest.fixture(scope="module")
def c1(c1_graph):
    g, _ = c1_graph
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    return g, val, x, y_ref, b


@pytest.mark.parametrize("mode", MODES)
def test_scale12_within_tolerance(ctx, c1, mode):
    g, val, x, y_ref, b = c1
    y = run(ctx, g, val, x, mode)
    assert oracle.spmv_check(y_ref, b, y) == (0, -1)


@pytest.mark.parametrize("mode", ["wave", "block", "grid"])
@pytest.mark.parametrize("tune", [dict(threshold=1), dict(threshold=2, block_threads=64), dict(threshold=500),
                                  dict(items_per_lane=1), dict(items_per_lane=16, block_threads=1024),
                                  dict(grid_blocks=2, block_threads=128)])
def test_tune_sweep_and_determinism(ctx, c1, mode, tune):
    g, val, x, y_ref, b = c1
    y1 = run(ctx, g, val, x, mode, **tune)
    y2 = run(ctx, g, val, x, mode, **tune)
    assert oracle.spmv_check(y_ref, b, y1) == (0, -1)
    assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))


@pytest.mark.parametrize("tune", [dict(threshold=8, items_per_lane=2), dict(threshold=1, items_per_lane=1),
                                  dict(threshold=32, items_per_lane=4), dict(threshold=3, items_per_lane=16)])
def test_same_order_in_every_consolidated_mode(ctx, c1, tune):
    """For a given threshold and items_per_lane, wave, block and grid modes sum
    each row in one order: rows up to the threshold by their own lane, rows up
    to one chunk (64 * items_per_lane) by the group of g = 2^ceil(log2(len /
    items_per_lane)) lanes, longer rows in chunks whose partials are combined in
    chunk order.  The workgroup size only moves rows between workgroups, so y
    is bitwise the same in the three modes at every block_threads, and flat
    mode (every row by its own lane) agrees on the rows up to the threshold."""
    g, val, x, y_ref, b = c1
    lens = np.diff(g.row_ptr)
    y0 = run(ctx, g, val, x, "grid", **tune)
    assert oracle.spmv_check(y_ref, b, y0) == (0, -1)
    for mode in ("wave", "block", "grid"):
        for bt in (64, 256, 1024):
            y = run(ctx, g, val, x, mode, block_threads=bt, **tune)
            assert np.array_equal(y.view(np.uint32), y0.view(np.uint32)), (mode, bt)
    light = lens <= tune["threshold"]
    assert light.any() and (~light).any()
    yf = run(ctx, g, val, x, "flat")
    assert np.array_equal(yf[light].view(np.uint32), y0[light].view(np.uint32))


@pytest.mark.parametrize("tune", [dict(threshold=8, items_per_lane=2), dict(threshold=1, items_per_lane=1),
                                  dict(threshold=32, items_per_lane=4)])
def test_row_lengths_at_every_boundary(ctx, tune):
    """Rows whose lengths sit on every boundary of the per-row order (the
    threshold, each lane-group size g * items_per_lane, the chunk of
    64 * items_per_lane and one past it), 40 rows of each length in shuffled
    order so that every window mixes them: within the bound in every mode and
    bitwise the same in wave, block and grid modes."""
    rng = np.random.default_rng(91)
    thr, ipl = tune["threshold"], tune["items_per_lane"]
    lens = {0, 1, thr, thr + 1, 64 * ipl - 1, 64 * ipl, 64 * ipl + 1, 2 * 64 * ipl + 1, 1000}
    for g in (1, 2, 4, 8, 16, 32, 64):
        lens |= {g * ipl, g * ipl + 1}
    row_lens = rng.permutation(np.repeat(sorted(x for x in lens if x >= 0), 40))
    n = len(row_lens)
    edges = [(r, int(c)) for r, ln in enumerate(row_lens) for c in rng.integers(0, n, ln)]
    g, _ = synth.graph_from_edges(n, edges)
    assert np.array_equal(np.diff(g.row_ptr), row_lens)
    val, x = synth.values(g.m, seed=92), synth.vector_x(n, seed=93)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    ys = {}
    for mode in MODES:
        ys[mode] = run(ctx, g, val, x, mode, **tune)
        assert oracle.spmv_check(y_ref, b, ys[mode]) == (0, -1), mode
    for mode in ("wave", "block"):
        assert np.array_equal(ys[mode].view(np.uint32), ys["grid"].view(np.uint32)), mode


@pytest.mark.parametrize("mode", MODES)
def test_edge_cases(ctx, mode):
    rng = np.random.default_rng(8)
    cases = []
    n = 1500
    cases.append(("identity", synth.graph_from_edges(n, [(i, i) for i in range(n)])[0]))
    cases.append(("empty_rows", synth.graph_from_edges(n, [(7, 3), (7, 9), (1000, 1)])[0]))
    cases.append(("one_huge_row", synth.graph_from_edges(n, [(3, j % n) for j in range(100000)])[0]))
    cases.append(("no_entries", synth.graph_from_edges(n, [])[0]))
    cases.append(("single", synth.graph_from_edges(1, [(0, 0)])[0]))
    e = list(zip(rng.integers(0, 300, 9000).tolist(), rng.integers(0, 300, 9000).tolist()))
    cases.append(("uniform", synth.graph_from_edges(300, e)[0]))
    for name, g in cases:
        val = synth.values(g.m, seed=31)
        x = synth.vector_x(g.n, seed=37)
        y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
        for tune in (dict(), dict(threshold=1), dict(threshold=1, items_per_lane=1)):
            y = run(ctx, g, val, x, mode, **tune)
            assert oracle.spmv_check(y_ref, b, y) == (0, -1), (name, tune)
            empty = np.diff(g.row_ptr) == 0
            assert (y[empty] == 0).all()


def test_bookkeeping_matches_oracle_plan(ctx, c1):
    g, val, x, y_ref, b = c1
    lens = np.diff(g.row_ptr).astype(np.int64)
    for t in (8, 32, 100):
        heavy = oracle.count_heavy(lens, t)
        _, st = run(ctx, g, val, x, "wave", stats=True, threshold=t)
        assert st["items_buffered"] == heavy
        assert st["dispatches"] == oracle.consolidation_plan(lens, t, 64)["dispatches"]
        assert st["edges_processed"] == g.m
        for bt in (128, 256):
            _, st = run(ctx, g, val, x, "block", stats=True, threshold=t, block_threads=bt)
            assert st["items_buffered"] == heavy
            assert st["dispatches"] == oracle.consolidation_plan(lens, t, bt)["dispatches"]
        _, st = run(ctx, g, val, x, "grid", stats=True, threshold=t)
        assert st["items_buffered"] == heavy and st["dispatches"] == (1 if heavy else 0)
        _, st = run(ctx, g, val, x, "flat", stats=True)
        assert st["items_buffered"] == 0 and st["dispatches"] == 0


def test_basic_driver_emulates_per_row_children(ctx, c1):
    """Driver 2 (basic dynamic parallelism emulated: one host-launched child per
    heavy row) gives the same bound and one child launch per row above the
    threshold; it is reproducible run to run."""
    g, val, x, y_ref, b = c1
    lens = np.diff(g.row_ptr)
    for th in (8, 64):
        y1, st = run(ctx, g, val, x, "grid", stats=True, driver=2, threshold=th)
        y2 = run(ctx, g, val, x, "grid", driver=2, threshold=th)
        assert oracle.spmv_check(y_ref, b, y1) == (0, -1)
        assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))
        assert st["dispatches"] == st["items_buffered"] == int((lens > th).sum())
    da = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    for mode, tune in (("block", dict(driver=2)), ("grid", dict(driver=3)), ("grid", dict(driver=1))):
        with pytest.raises(wc.WcError):
            ctx.spmv(da, f32_to_dev(val), f32_to_dev(x), mode=mode, tune=wc.make_tune(**tune))
    torch.cuda.synchronize()


def test_fig2_worked_example(ctx):
    """Two heavy rows of 326 and 234 nonzeros in one scope: one consolidated
    dispatch carrying both (Sec. IV.A, Fig. 2)."""
    lens = [3, 326, 5, 7, 234, 2, 1, 8]
    n = 400
    edges = [(r, j % n) for r, ln in enumerate(lens) for j in range(ln)]
    g, _ = synth.graph_from_edges(n, edges)
    val, x = synth.values(g.m, seed=5), synth.vector_x(n, seed=6)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    plan = oracle.consolidation_plan(np.diff(g.row_ptr), 64, n)
    assert plan["basic_launches"] == 2 and plan["total_work"] == 560
    for mode in ("wave", "block", "grid"):
        y, st = run(ctx, g, val, x, mode, stats=True, threshold=64)
        assert oracle.spmv_check(y_ref, b, y) == (0, -1)
        assert st["items_buffered"] == 2 and st["dispatches"] == 1


def test_grid_overflow(ctx, c1):
    g, val, x, y_ref, b = c1
    y, st = run(ctx, g, val, x, "grid", stats=True, threshold=4, buf_capacity=7)
    assert st["overflowed"] == 1 and oracle.spmv_check(y_ref, b, y) == (0, -1)
    with pytest.raises(wc.WcError):
        run(ctx, g, val, x, "grid", stats=True, threshold=4, buf_capacity=7, allow_fallback=-1)


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_long_rows_handed_to_the_grid(ctx, c1, mode):
    """Rows longer than one group's child can take (one chunk of
    64 * items_per_lane nonzeros) go to the global chunks that the grid-wide
    drain sums: same bound, bitwise reproducible, the same rows
    counted as buffered, and an undersized buffer falls back to the row's lane
    (overflow flag; WC_EOVERFLOW when the fallback is refused)."""
    g, val, x, y_ref, b = c1
    lens = np.diff(g.row_ptr)
    for tune in (dict(), dict(items_per_lane=1), dict(items_per_lane=1, block_threads=64),
                 dict(items_per_lane=2, threshold=2)):
        ipl, bt = tune.get("items_per_lane", 2), tune.get("block_threads", 256)
        spill = 64 * ipl
        assert (lens > spill).any()
        y1, st = run(ctx, g, val, x, mode, stats=True, **tune)
        y2 = run(ctx, g, val, x, mode, **tune)
        assert oracle.spmv_check(y_ref, b, y1) == (0, -1), tune
        assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32)), tune
        assert st["items_buffered"] == oracle.count_heavy(lens, tune.get("threshold", 8))
        assert st["overflowed"] == 0
    y, st = run(ctx, g, val, x, mode, stats=True, items_per_lane=1, buf_capacity=5)
    assert st["overflowed"] == 1 and oracle.spmv_check(y_ref, b, y) == (0, -1)
    with pytest.raises(wc.WcError) as ei:
        run(ctx, g, val, x, mode, stats=True, items_per_lane=1, buf_capacity=5, allow_fallback=-1)
    assert ei.value.status == -3


@pytest.fixture(scope="module")
def c2_spmv():
    say("generating scale-22 matrix")
    g = synth.rmat_csr(22, 1 << 26)
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    return g, val, x, y_ref, b


@pytest.mark.parametrize("mode", MODES)
def test_scale22_within_tolerance(ctx, c2_spmv, mode):
    g, val, x, y_ref, b = c2_spmv
    y = run(ctx, g, val, x, mode)
    assert oracle.spmv_check(y_ref, b, y) == (0, -1)
