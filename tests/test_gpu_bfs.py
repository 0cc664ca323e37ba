"""GPU parity of wc_bfs against the oracle's breadth-first levels, bit-exact in
every mode and tune: flat and grid modes run the frontier rounds of the SSSP
path with unit weights, wave and block modes the recursion path (recursive
calls consolidated into per-group packets of a device queue).  Special graphs,
argument errors, a call list too small for the recursion path (recomputed by
the rounds, overflow flag), the timeout path, and the scale-22 graph
(certificate + exact)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def run(ctx, dg, src, mode, **tune):
    t = wc.make_tune(**tune) if tune else None
    lv = ctx.bfs(dg, src, mode=mode, tune=t)
    torch.cuda.synchronize()
    return dev_to_u32(lv)


@pytest.mark.parametrize("mode", MODES)
def test_scale12_sources_and_tunes(ctx, c1_graph, mode):
    g, _ = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    for src in (0, 1, 77, g.n - 1):
        say(f"bfs scale 12 mode={mode} src={src}")
        assert np.array_equal(run(ctx, dg, src, mode), oracle.bfs(g.row_ptr, g.col, src)), src
    ref = oracle.bfs(g.row_ptr, g.col, 0)
    for tune in (dict(threshold=1), dict(block_threads=64, items_per_lane=1), dict(block_threads=1024),
                 dict(grid_blocks=2), dict(items_per_lane=16), dict(grid_blocks=1, block_threads=64)):
        assert np.array_equal(run(ctx, dg, 0, mode, **tune), ref), tune


def shapes():
    yield "single", synth.graph_from_edges(1, [])[0]
    yield "path", synth.graph_from_edges(2000, [(i, i + 1) for i in range(1999)])[0]
    yield "star_out", synth.graph_from_edges(5000, [(0, i) for i in range(1, 5000)])[0]
    yield "two_components", synth.graph_from_edges(10, [(0, 1), (1, 2), (5, 6)])[0]
    # a long path with shortcuts: calls made at a too-deep level go stale
    e = [(i, i + 1) for i in range(2999)] + [(0, 1500), (1500, 2999), (10, 2000)]
    yield "path_with_shortcuts", synth.graph_from_edges(3000, e)[0]
    hub = [(0, i) for i in range(1, 20000)] + [(i, (i * 7) % 20000) for i in range(1, 20000)]
    yield "hub_and_ring", synth.graph_from_edges(20000, hub)[0]
    yield "self_and_multi", synth.graph_from_edges(4, [(0, 0), (0, 1), (0, 1), (1, 3), (3, 1)])[0]


@pytest.mark.parametrize("mode", MODES)
def test_shapes(ctx, mode):
    for name, g in shapes():
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        assert np.array_equal(run(ctx, dg, 0, mode), oracle.bfs(g.row_ptr, g.col, 0)), name


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_recursion_path_bookkeeping_and_overflow(ctx, c1_graph, mode):
    """Wave and block modes: every reached vertex with out-edges is a recursive
    call at least once (entries >= such vertices, packets >= 1, improvements >=
    reached - 1); a call list too small falls back to the frontier rounds with
    the same levels and the overflow flag (WC_EOVERFLOW if refused)."""
    g, _ = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    ref = oracle.bfs(g.row_ptr, g.col, 0)
    reached = ref != np.uint32(0xFFFFFFFF)
    calls = int((reached & (np.diff(g.row_ptr) > 0)).sum())
    lv, st = ctx.bfs(dg, 0, mode=mode, stats=True)
    assert np.array_equal(dev_to_u32(lv), ref)
    assert st["overflowed"] == 0 and st["items_buffered"] >= calls and st["dispatches"] >= 1
    assert st["updates"] >= int(reached.sum()) - 1
    lv, st = ctx.bfs(dg, 0, mode=mode, tune=wc.make_tune(buf_capacity=50), stats=True)
    assert np.array_equal(dev_to_u32(lv), ref) and st["overflowed"] == 1
    with pytest.raises(wc.WcError) as ei:
        ctx.bfs(dg, 0, mode=mode, tune=wc.make_tune(buf_capacity=50, allow_fallback=-1))
    assert ei.value.status == -3
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_recursion_path_timeout_is_reported(c1_graph, mode):
    """A wait for packets bounded at 1 microsecond gives up (every kernel still
    ends normally) and the call reports WC_ETIMEOUT; a later call with the
    default bound is exact again."""
    g, _ = c1_graph
    c = wc.Context(0)
    try:
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        c.set_wait_limit(1)
        timed_out = 0
        for _ in range(5):
            try:
                c.bfs(dg, 0, mode=mode)
            except wc.WcError as e:
                assert e.status == -4
                timed_out += 1
        torch.cuda.synchronize()
        assert timed_out >= 1
        c.set_wait_limit(0)
        assert np.array_equal(run(c, dg, 0, mode), oracle.bfs(g.row_ptr, g.col, 0))
    finally:
        c.close()


def test_invalid_arguments(ctx, c1_graph):
    g, _ = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, g.n)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, -1)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, 0, mode=5)
    for mode, tune in (("wave", dict(driver=2)), ("block", dict(buffer_alloc=1))):
        with pytest.raises(wc.WcError):
            ctx.bfs(dg, 0, mode=mode, tune=wc.make_tune(**tune))


@pytest.fixture(scope="module")
def c2_bfs():
    say("generating scale-22 graph for BFS")
    g = synth.rmat_csr(22, 1 << 26)
    return g, wc.DeviceCSR.from_host(g.row_ptr, g.col), oracle.bfs(g.row_ptr, g.col, 0)


@pytest.mark.parametrize("mode", MODES)
def test_scale22(ctx, c2_bfs, mode):
    g, dg, ref = c2_bfs
    say(f"bfs scale 22 mode={mode}")
    got = run(ctx, dg, 0, mode)
    assert np.array_equal(got, ref)
    assert oracle.sssp_certify(g.row_ptr, g.col, np.ones(len(g.col), np.uint32), 0, got) == (0, -1)
