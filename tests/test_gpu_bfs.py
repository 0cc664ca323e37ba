"""GPU parity of wc_bfs (recursive BFS on the SSSP kernels with unit weights):
bit-exact against the oracle's levels in every mode and tune, special graphs,
argument errors, and the scale-22 graph (certificate + exact)."""
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
                 dict(grid_blocks=2)):
        assert np.array_equal(run(ctx, dg, 0, mode, **tune), ref), tune


def shapes():
    yield "single", synth.graph_from_edges(1, [])[0]
    yield "path", synth.graph_from_edges(2000, [(i, i + 1) for i in range(1999)])[0]
    yield "star_out", synth.graph_from_edges(5000, [(0, i) for i in range(1, 5000)])[0]
    yield "two_components", synth.graph_from_edges(10, [(0, 1), (1, 2), (5, 6)])[0]
    yield "self_and_multi", synth.graph_from_edges(4, [(0, 0), (0, 1), (0, 1), (1, 3), (3, 1)])[0]


@pytest.mark.parametrize("mode", MODES)
def test_shapes(ctx, mode):
    for name, g in shapes():
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        assert np.array_equal(run(ctx, dg, 0, mode), oracle.bfs(g.row_ptr, g.col, 0)), name


def test_invalid_arguments(ctx, c1_graph):
    g, _ = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, g.n)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, -1)
    with pytest.raises(wc.WcError):
        ctx.bfs(dg, 0, mode=5)


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
