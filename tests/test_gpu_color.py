"""GPU parity of wc_color (Jones-Plassmann coloring, the GC benchmark): bit-exact
against the oracle's rounds in every mode and tune, the number of colors in the
stats, special graphs, buffer overflow, argument errors, a graph shaped like
the paper's Kron_log16 input, and the scale-22 graph (certificate: the
recurrence fixes every color, so zero violations means equal to the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say, u32_to_dev
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def sym(n, edges):
    return synth.symmetrize(synth.graph_from_edges(n, edges)[0])


def run(ctx, dg, dp, mode, stats=False, **tune):
    t = wc.make_tune(**tune) if tune else None
    out = ctx.color(dg, dp, mode=mode, tune=t, stats=stats)
    torch.cuda.synchronize()
    if stats:
        return out[0].cpu().numpy(), out[1]
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def c1_sym(c1_graph):
    g = synth.symmetrize(c1_graph[0])
    p = synth.priorities(g.n)
    return g, p, wc.DeviceCSR.from_host(g.row_ptr, g.col), u32_to_dev(p), oracle.color_jp(g.row_ptr, g.col, p)


@pytest.mark.parametrize("mode", MODES)
def test_scale12_exact_and_tunes(ctx, c1_sym, mode):
    g, p, dg, dp, (ref, k) = c1_sym
    say(f"color scale 12 mode={mode}")
    got, st = run(ctx, dg, dp, mode, stats=True)
    assert np.array_equal(got, ref)
    assert st["rounds"] == k and st["overflowed"] == 0
    assert st["edges_processed"] > 0
    if mode != "flat":
        assert st["edges_buffered"] > 0 and st["items_buffered"] > 0
    for tune in (dict(threshold=1), dict(threshold=1000), dict(block_threads=64, items_per_lane=1),
                 dict(block_threads=1024), dict(grid_blocks=2), dict(items_per_lane=64)):
        assert np.array_equal(run(ctx, dg, dp, mode, **tune), ref), tune


def test_priority_streams(ctx, c1_sym):
    g, _, dg, _, _ = c1_sym
    for stream in (601, 602):
        p = synth.priorities(g.n, stream=stream)
        ref, _ = oracle.color_jp(g.row_ptr, g.col, p)
        for mode in MODES:
            assert np.array_equal(run(ctx, dg, u32_to_dev(p), mode), ref), (stream, mode)


def shapes():
    yield "single", sym(1, []), np.array([3], np.uint32)
    yield "no_edges", sym(6, []), np.arange(6, dtype=np.uint32)
    k = 9
    yield "complete", sym(k, [(i, j) for i in range(k) for j in range(i + 1, k)]), synth.priorities(k)
    yield "star_hub_first", sym(5000, [(0, i) for i in range(1, 5000)]), \
        np.concatenate([[10 ** 9], np.arange(1, 5000)]).astype(np.uint32)
    yield "star_hub_last", sym(5000, [(0, i) for i in range(1, 5000)]), \
        np.concatenate([[0], np.arange(1, 5000)]).astype(np.uint32)
    # increasing priorities along a path: one vertex per round, 700 rounds
    yield "path_increasing", sym(700, [(i, i + 1) for i in range(699)]), np.arange(700, dtype=np.uint32)
    yield "equal_priorities", synth.symmetrize(synth.rmat_csr(10, 1 << 13)), np.zeros(1 << 10, np.uint32)
    yield "self_and_multi", synth.graph_from_edges(4, [(0, 0), (0, 1), (1, 0), (0, 1), (1, 0), (1, 3), (3, 1)])[0], \
        np.array([1, 2, 3, 4], np.uint32)
    # a hub whose neighbours carry the largest priorities, and another graph component
    hub = [(0, i) for i in range(1, 3000)] + [(3000 + i, 3001 + i) for i in range(500)]
    yield "hub_plus_path", sym(3501, hub), synth.priorities(3501, stream=603)


@pytest.mark.parametrize("mode", MODES)
def test_shapes(ctx, mode):
    for name, g, p in shapes():
        say(f"color shape {name} mode={mode}")
        ref, k = oracle.color_jp(g.row_ptr, g.col, p)
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        got, st = run(ctx, dg, u32_to_dev(p), mode, stats=True)
        assert np.array_equal(got, ref), name
        assert st["rounds"] == k, name
        got = run(ctx, dg, u32_to_dev(p), mode, threshold=1, block_threads=64)
        assert np.array_equal(got, ref), name


def test_empty_graph(ctx):
    dg = wc.DeviceCSR.from_host(np.zeros(1, np.int32), np.zeros(0, np.int32))
    out = torch.empty(0, dtype=torch.int32, device="cuda")
    got, st = ctx.color(dg, torch.empty(0, dtype=torch.int32, device="cuda"), out=out, stats=True)
    assert got.numel() == 0 and st["rounds"] == 0


def test_buffer_overflow(ctx, c1_sym):
    g, p, dg, dp, (ref, _) = c1_sym
    got, st = run(ctx, dg, dp, "grid", stats=True, threshold=1, buf_capacity=5)
    assert np.array_equal(got, ref) and st["overflowed"] == 1
    with pytest.raises(wc.WcError):
        ctx.color(dg, dp, mode="grid", tune=wc.make_tune(threshold=1, buf_capacity=5, allow_fallback=-1))
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_long_ranges_handed_to_the_grid(ctx, c1_sym, mode):
    """Wave and block modes hand every buffered vertex with more than one chunk
    (64 * items_per_lane) of neighbours on to a grid-wide drain, in the count
    pass and in every round: exact for several chunk sizes and workgroup
    sizes, and an undersized buffer falls back to the vertex's own lane
    (overflow flag; WC_EOVERFLOW when the fallback is refused)."""
    g, p, dg, dp, (ref, k) = c1_sym
    deg = np.diff(g.row_ptr)
    for tune in (dict(), dict(items_per_lane=4), dict(items_per_lane=1, block_threads=64),
                 dict(items_per_lane=2, threshold=2), dict(items_per_lane=1, block_threads=1024)):
        assert (deg > 64 * tune.get("items_per_lane", 1)).any()
        got, st = run(ctx, dg, dp, mode, stats=True, **tune)
        assert np.array_equal(got, ref), tune
        assert st["rounds"] == k and st["overflowed"] == 0, tune
    got, st = run(ctx, dg, dp, mode, stats=True, items_per_lane=1, buf_capacity=3)
    assert np.array_equal(got, ref) and st["overflowed"] == 1
    with pytest.raises(wc.WcError) as ei:
        ctx.color(dg, dp, mode=mode, tune=wc.make_tune(items_per_lane=1, buf_capacity=3, allow_fallback=-1))
    assert ei.value.status == -3
    torch.cuda.synchronize()


def test_invalid_arguments(ctx, c1_sym):
    g, p, dg, dp, _ = c1_sym
    with pytest.raises(wc.WcError):
        ctx.color(dg, dp, mode=5)
    for driver in (1, 2, 3):
        with pytest.raises(wc.WcError):
            ctx.color(dg, dp, mode="grid", tune=wc.make_tune(driver=driver))
    with pytest.raises(ValueError):
        ctx.color(dg, dp[:-1])


def test_asymmetric_graph_is_rejected(ctx):
    # 1 outranks 0 but has no edge back: 0 is never released
    g, _ = synth.graph_from_edges(2, [(0, 1)])
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    with pytest.raises(wc.WcError):
        ctx.color(dg, u32_to_dev(np.array([0, 5], np.uint32)))
    torch.cuda.synchronize()
    # the library stays usable after the error
    g = sym(3, [(0, 1), (1, 2)])
    got = ctx.color(wc.DeviceCSR.from_host(g.row_ptr, g.col), u32_to_dev(np.array([0, 1, 2], np.uint32)))
    assert got.cpu().numpy().tolist() == [2, 1, 0]


@pytest.fixture(scope="module")
def kron16():
    """Scale-16 R-MAT, symmetrized (about 4M directed edges, like Kron_log16)."""
    g = synth.symmetrize(synth.rmat_csr(16, 1 << 21))
    p = synth.priorities(g.n)
    return g, p, wc.DeviceCSR.from_host(g.row_ptr, g.col), u32_to_dev(p), oracle.color_jp(g.row_ptr, g.col, p)


@pytest.mark.parametrize("mode", MODES)
def test_kron16_exact(ctx, kron16, mode):
    g, p, dg, dp, (ref, k) = kron16
    say(f"color kron16 mode={mode} colors={k}")
    got, st = run(ctx, dg, dp, mode, stats=True)
    assert np.array_equal(got, ref) and st["rounds"] == k
    # repeated calls give the same colors (no state kept between calls)
    assert np.array_equal(run(ctx, dg, dp, mode), ref)


@pytest.fixture(scope="module")
def c2_sym():
    say("generating symmetrized scale-22 graph for coloring")
    g = synth.symmetrize(synth.rmat_csr(22, 1 << 26))
    p = synth.priorities(g.n)
    return g, p, wc.DeviceCSR.from_host(g.row_ptr, g.col), u32_to_dev(p)


@pytest.mark.parametrize("mode", ["wave", "block", "grid"])
def test_scale22_certified(ctx, c2_sym, mode):
    g, p, dg, dp = c2_sym
    say(f"color scale 22 mode={mode}")
    got, st = run(ctx, dg, dp, mode, stats=True)
    assert oracle.color_certify(g.row_ptr, g.col, p, got) == (0, -1)
    assert st["rounds"] == int(got.max()) + 1
