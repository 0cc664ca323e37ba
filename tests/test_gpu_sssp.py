"""GPU parity of wc_sssp against the oracle (bit-exact distances).

Every mode on the scale-12 R-MAT graph, launch-configuration sweeps, both
drivers, adversarial shapes, forced buffer overflow, repeat runs, and the
scale-22 graph (full comparison with Dijkstra plus the optimality certificate).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, say, u32_to_dev
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def upload(g, w):
    return wc.DeviceCSR.from_host(g.row_ptr, g.col), u32_to_dev(w)


def run(ctx, g, w, src, mode, **tune):
    dg, dw = upload(g, w)
    t = wc.make_tune(**tune) if tune else None
    say(f"sssp n={g.n} m={g.m} src={src} mode={mode} tune={tune}")
    d = ctx.sssp(dg, dw, src, mode=mode, tune=t)
    torch.cuda.synchronize()
    return dev_to_u32(d)


@pytest.fixture(scope="module")
def c1(c1_graph):
    g, w = c1_graph
    return g, w, oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)


@pytest.mark.parametrize("mode", MODES)
def test_scale12_all_modes_bit_exact(ctx, c1, mode):
    g, w, ref = c1
    assert np.array_equal(run(ctx, g, w, 0, mode), ref)


@pytest.mark.parametrize("mode", ["wave", "block", "grid"])
@pytest.mark.parametrize("tune", [dict(threshold=1), dict(threshold=8, block_threads=64),
                                  dict(threshold=100, block_threads=1024), dict(items_per_lane=1),
                                  dict(items_per_lane=16, block_threads=128), dict(grid_blocks=3),
                                  dict(threshold=2, block_threads=512)])
def test_scale12_tune_sweep(ctx, c1, mode, tune):
    g, w, ref = c1
    assert np.array_equal(run(ctx, g, w, 0, mode, **tune), ref)


@pytest.mark.parametrize("mode", MODES)
def test_other_sources_and_seeds(ctx, mode):
    g = synth.rmat_csr(11, 1 << 15, seed=17)
    w = synth.weights(g.m, seed=23)
    deg = g.degrees()
    for src in (1, int(np.argmax(deg)), int(np.flatnonzero(deg == 0)[0]), g.n - 1):
        ref = oracle.sssp_dijkstra(g.row_ptr, g.col, w, src)
        assert np.array_equal(run(ctx, g, w, src, mode, threshold=4), ref)


def shapes():
    n = 3000
    yield "star_out", synth.graph_from_edges(n, [(0, i) for i in range(1, n)], np.arange(1, n) % 100 + 1)
    yield "star_in", synth.graph_from_edges(n, [(0, 1)] + [(i, 0) for i in range(1, n)] +
                                            [(1, i) for i in range(2, n)], None)
    yield "chain", synth.graph_from_edges(500, [(i, i + 1) for i in range(499)], np.arange(499) % 7 + 1)
    rng = np.random.default_rng(4)
    e = [(int(a), int(b)) for a, b in zip(rng.integers(0, 500, 4000), rng.integers(0, 500, 4000))]
    yield "uniform", synth.graph_from_edges(500, e, rng.integers(1, 101, 4000))
    yield "no_edges", synth.graph_from_edges(10, [], [])
    yield "single", synth.graph_from_edges(1, [], [])
    yield "self_loops", synth.graph_from_edges(4, [(0, 0), (0, 1), (1, 1), (1, 2), (2, 0)], [3, 2, 1, 5, 1])
    # many hubs in one window plus parallel edges (multi-edges)
    hub = [(i, j) for i in range(8) for j in range(8, 2000)] + [(5, 9)] * 50
    yield "hubs", synth.graph_from_edges(2000, hub, (np.arange(len(hub)) % 100) + 1)


@pytest.mark.parametrize("mode", MODES)
def test_adversarial_shapes(ctx, mode):
    for name, (g, w) in shapes():
        w = np.asarray(w, dtype=np.uint32)
        ref = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
        for tune in (dict(), dict(threshold=1), dict(block_threads=64, items_per_lane=1)):
            got = run(ctx, g, w, 0, mode, **tune)
            assert np.array_equal(got, ref), (name, tune)


def test_grid_overflow_falls_back_and_can_fail(ctx, c1):
    g, w, ref = c1
    dg, dw = upload(g, w)
    d, st = ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(threshold=1, buf_capacity=5), stats=True)
    assert np.array_equal(dev_to_u32(d), ref) and st["overflowed"] == 1
    with pytest.raises(wc.WcError) as ei:
        ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(threshold=1, buf_capacity=5, allow_fallback=-1),
                 stats=True)
    assert ei.value.status == -3
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_long_items_handed_to_the_grid(ctx, c1, mode):
    """Vertices with more edges than one group's child keeps (one chunk of
    64 * items_per_lane edges) are handed on to the grid-wide drain of the
    round: identical distances for several chunk sizes, and an undersized
    buffer falls back to the writing lanes (overflow flag; WC_EOVERFLOW when the
    fallback is refused)."""
    g, w, ref = c1
    dg, dw = upload(g, w)
    deg = np.diff(g.row_ptr)
    for tune in (dict(), dict(items_per_lane=1), dict(items_per_lane=1, block_threads=64), dict(threshold=2)):
        ipl, bt = tune.get("items_per_lane", 2), tune.get("block_threads", 256)
        spill = 64 * ipl
        assert (deg > spill).any()
        d, st = ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(**tune), stats=True)
        assert np.array_equal(dev_to_u32(d), ref), tune
        assert st["overflowed"] == 0 and st["updates_buffered"] >= 1
    d, st = ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(items_per_lane=1, buf_capacity=3), stats=True)
    assert np.array_equal(dev_to_u32(d), ref) and st["overflowed"] == 1
    with pytest.raises(wc.WcError) as ei:
        ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(items_per_lane=1, buf_capacity=3, allow_fallback=-1),
                 stats=True)
    assert ei.value.status == -3


@pytest.mark.parametrize("mode", ["wave", "block"])
@pytest.mark.parametrize("alloc", [1, 2])
def test_group_buffers_in_global_memory(ctx, c1, mode, alloc):
    """The allocator comparison (Sec. V.A): each wave's or block's buffer in a
    slice of the pre-allocated pool (1) or from device-side malloc, freed after
    the child (2), instead of registers / LDS; identical distances (a malloc
    that fails keeps the items in registers / LDS and only raises the flag)."""
    g, w, ref = c1
    dg, dw = upload(g, w)
    for tune in (dict(), dict(threshold=1, block_threads=64), dict(block_threads=1024, items_per_lane=1)):
        say(f"sssp buffer_alloc={alloc} mode={mode} tune={tune}")
        d, st = ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(buffer_alloc=alloc, **tune), stats=True)
        assert np.array_equal(dev_to_u32(d), ref), tune
        if alloc == 1:
            assert st["overflowed"] == 0


def test_buffer_alloc_is_refused_where_it_does_not_apply(ctx, c1):
    g, w, _ = c1
    dg, dw = upload(g, w)
    for mode, alloc in (("grid", 1), ("flat", 2), ("wave", 3), ("block", -1)):
        with pytest.raises(wc.WcError) as ei:
            ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(buffer_alloc=alloc))
        assert ei.value.status == -1
    with pytest.raises(wc.WcError):
        ctx.spmv(dg, torch.zeros(g.m, device="cuda"), torch.zeros(g.n, device="cuda"), mode="wave",
                 tune=wc.make_tune(buffer_alloc=1))
    torch.cuda.synchronize()


def test_persistent_driver_is_refused(ctx, c1):
    """The persistent co-resident driver is switched off (it hung in block mode
    and no cause has been shown); asking for it is an argument error."""
    g, w, _ = c1
    dg, dw = upload(g, w)
    with pytest.raises(wc.WcError) as ei:
        ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(driver=1))
    assert ei.value.status == -1


def test_basic_driver_emulates_per_vertex_children(ctx, c1):
    """driver = 2: one host-launched child per buffered vertex (the unconsolidated
    basic-dp baseline); same distances, and one dispatch per heavy expansion."""
    g, w, ref = c1
    dg, dw = upload(g, w)
    d, st = ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(driver=2), stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(dev_to_u32(d), ref)
    assert st["dispatches"] == st["items_buffered"] >= 1
    for mode in ("flat", "wave", "block"):
        with pytest.raises(wc.WcError):
            ctx.sssp(dg, dw, 0, mode=mode, tune=wc.make_tune(driver=2))
    with pytest.raises(wc.WcError):
        ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(driver=4))


def test_one_to_one_mapped_child(ctx, c1):
    """driver = 3: the drain launched with one wave per buffered chunk."""
    g, w, ref = c1
    dg, dw = upload(g, w)
    for tune in (dict(driver=3), dict(driver=3, block_threads=64, items_per_lane=1)):
        d = ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(**tune))
        torch.cuda.synchronize()
        assert np.array_equal(dev_to_u32(d), ref), tune
    with pytest.raises(wc.WcError):
        ctx.sssp(dg, dw, 0, mode="block", tune=wc.make_tune(driver=3))


def test_invalid_arguments(ctx, c1):
    g, w, _ = c1
    dg, dw = upload(g, w)
    for bad in (-1, g.n):
        with pytest.raises(wc.WcError) as ei:
            ctx.sssp(dg, dw, bad, mode="grid")
        assert ei.value.status == -1
    with pytest.raises(wc.WcError):
        ctx.sssp(dg, dw, 0, mode=7)
    with pytest.raises(wc.WcError):
        ctx.sssp(dg, dw, 0, mode="grid", tune=wc.make_tune(block_threads=96))


def test_stats_and_repeat_runs(ctx, c1):
    g, w, ref = c1
    dg, dw = upload(g, w)
    reached = oracle.sssp_reached_edges(g.row_ptr, ref)
    n_reached = int((ref != np.uint32(0xFFFFFFFF)).sum())
    for mode in MODES:
        for _ in range(10):
            d, st = ctx.sssp(dg, dw, 0, mode=mode, stats=True)
            assert np.array_equal(dev_to_u32(d), ref)
            assert st["rounds"] >= 1 and st["edges_processed"] >= reached
            # every reached vertex but the source was lowered from infinity at least once
            assert n_reached - 1 <= st["updates"] <= st["edges_processed"]
            assert 0 <= st["updates_buffered"] <= st["updates"]
            assert (st["updates_buffered"] == 0) == (mode == "flat")
            if mode == "flat":
                assert st["items_buffered"] == 0 and st["dispatches"] == 0
            else:
                assert st["items_buffered"] >= 1 and st["dispatches"] >= 1


def test_kernel_timing_records(ctx, c1):
    """Per-kernel timing: one record per launch, in launch order, with positive
    durations that tile the call (their sum stays within the call's own elapsed
    time), aggregates that match the records, and unchanged results."""
    g, w, ref = c1
    dg, dw = upload(g, w)
    d = ctx.sssp(dg, dw, 0, mode="grid")
    torch.cuda.synchronize()
    ctx.set_timing(True)
    try:
        for rep in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            d = ctx.sssp(dg, dw, 0, mode="grid", out=d)
            b.record()
            torch.cuda.synchronize()
            assert np.array_equal(dev_to_u32(d), ref)
            recs = ctx.kernel_records()
            names = [n for n, _ in recs]
            assert names[:2] == ["zero_stats", "sssp_init"]
            body = names[2:]
            assert len(body) % 2 == 0 and body[0::2] == ["sssp_round_grid"] * (len(body) // 2)
            assert body[1::2] == ["sssp_drain"] * (len(body) // 2)
            assert all(ms > 0 for _, ms in recs)
            assert sum(ms for _, ms in recs) <= a.elapsed_time(b) * 1.02 + 0.01
            kt = ctx.kernel_times()
            assert kt["sssp_drain"][0] == len(body) // 2
            assert abs(kt["sssp_drain"][1] - sum(ms for n, ms in recs if n == "sssp_drain")) < 1e-6
            ctx.set_timing(True)  # discards the records
    finally:
        ctx.set_timing(False)


@pytest.fixture(scope="module")
def c2_sssp():
    say("generating scale-22 graph")
    g = synth.rmat_csr(22, 1 << 26)
    w = synth.weights(g.m)
    say("oracle Dijkstra at scale 22")
    ref = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    return g, w, ref


@pytest.mark.parametrize("mode", MODES)
def test_scale22_bit_exact(ctx, c2_sssp, mode):
    g, w, ref = c2_sssp
    got = run(ctx, g, w, 0, mode)
    assert np.array_equal(got, ref)
    assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, got) == (0, -1)
