"""GPU parity of wc_pagerank against the binary64 oracle, every mode and tune,
bit-identical repeats, special graphs, argument errors, and the scale-22 graph.
The relative bound per vertex is derived for each mode, tune and number of
sweeps from the rounding depth of the kernels' sums (tests/tolerance.py)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say
from paper_1606_08150_amd import wc
from tolerance import pagerank_rtol

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def upload(g):
    t = synth.transpose(g)
    return (wc.DeviceCSR.from_host(t.row_ptr, t.col), torch.from_numpy(synth.out_degree(g)).cuda(), t)


def reference(g, t, iters, d=0.85):
    return oracle.pagerank_f64(t.row_ptr, t.col, synth.out_degree(g), iters, d)


def bound(t, iters, mode, **tune):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return pagerank_rtol(iters, np.diff(t.row_ptr), mode, t.n, num_cus=cus, **tune)


@pytest.fixture(scope="module")
def c1_pr(c1_graph):
    g, _ = c1_graph
    dg, od, t = upload(g)
    return g, dg, od, t, {k: reference(g, t, k) for k in (0, 1, 10, 30)}


@pytest.mark.parametrize("mode", MODES)
def test_scale12_all_modes(ctx, c1_pr, mode):
    g, dg, od, t, refs = c1_pr
    for k, ref in refs.items():
        say(f"pagerank scale 12 mode={mode} iterations={k}")
        r = ctx.pagerank(dg, od, k, mode=mode)
        torch.cuda.synchronize()
        got = r.cpu().numpy()
        assert oracle.pagerank_check(ref, got, bound(t, k, mode)) == (0, -1), k
        assert abs(float(got.astype(np.float64).sum()) - 1.0) < 1e-4


@pytest.mark.parametrize("mode", ["block", "grid"])
@pytest.mark.parametrize("tune", [dict(threshold=1), dict(threshold=100), dict(items_per_lane=1),
                                  dict(items_per_lane=16), dict(block_threads=64), dict(block_threads=1024),
                                  dict(grid_blocks=3)])
def test_tune_sweep_and_repeats(ctx, c1_pr, mode, tune):
    g, dg, od, t, refs = c1_pr
    tt = wc.make_tune(**tune)
    first = ctx.pagerank(dg, od, 10, mode=mode, tune=tt).cpu().numpy()
    assert oracle.pagerank_check(refs[10], first, bound(t, 10, mode, **tune)) == (0, -1)
    for _ in range(3):
        again = ctx.pagerank(dg, od, 10, mode=mode, tune=tt).cpu().numpy()
        assert np.array_equal(again.view(np.uint32), first.view(np.uint32))


def test_same_order_in_every_consolidated_mode(ctx, c1_pr):
    """The in-edge sums follow one order per (threshold, items_per_lane) in
    wave, block and grid modes (as for SpMV) and the per-sweep kernels do not
    depend on the mode, so ten sweeps give bitwise the same ranks in the three
    modes, within the bound of each."""
    g, dg, od, t, refs = c1_pr
    for tune in (dict(threshold=8, items_per_lane=2), dict(threshold=2, items_per_lane=8)):
        tt = wc.make_tune(**tune)
        ranks = {m: ctx.pagerank(dg, od, 10, mode=m, tune=tt).cpu().numpy() for m in ("wave", "block", "grid")}
        for m, r in ranks.items():
            assert oracle.pagerank_check(refs[10], r, bound(t, 10, m, **tune)) == (0, -1), (m, tune)
            assert np.array_equal(r.view(np.uint32), ranks["grid"].view(np.uint32)), (m, tune)


def test_grid_sweeps_reuse_the_first_binning(ctx, c1_pr):
    """Grid mode bins the in-edge rows in the first sweep and reuses the binned
    rows and chunks in the later ones (full-size buffers, no work counters):
    the ranks are bitwise those of the path that bins every sweep (a buffer
    capacity given, or work counters on), for several tunes and sweep counts."""
    g, dg, od, t, refs = c1_pr
    for tune in (dict(), dict(threshold=1, items_per_lane=1), dict(block_threads=1024, items_per_lane=2)):
        for k in (1, 2, 10):
            reuse = ctx.pagerank(dg, od, k, mode="grid", tune=wc.make_tune(**tune) if tune else None)
            rebin = ctx.pagerank(dg, od, k, mode="grid", tune=wc.make_tune(buf_capacity=1 << 40, **tune))
            counted, _ = ctx.pagerank(dg, od, k, mode="grid", tune=wc.make_tune(**tune) if tune else None, stats=True)
            torch.cuda.synchronize()
            r0 = reuse.cpu().numpy()
            assert oracle.pagerank_check(refs[10] if k == 10 else reference(g, t, k), r0,
                                         bound(t, k, "grid", **tune)) == (0, -1), (tune, k)
            for other in (rebin, counted):
                assert np.array_equal(other.cpu().numpy().view(np.uint32), r0.view(np.uint32)), (tune, k)


def special_graphs():
    yield "single", synth.graph_from_edges(1, [])[0]
    yield "no_edges", synth.graph_from_edges(50, [])[0]
    yield "cycle", synth.graph_from_edges(9, [(i, (i + 1) % 9) for i in range(9)])[0]
    yield "star_in", synth.graph_from_edges(3000, [(i, 0) for i in range(1, 3000)])[0]
    yield "star_out", synth.graph_from_edges(3000, [(0, i) for i in range(1, 3000)])[0]
    yield "self_and_multi", synth.graph_from_edges(5, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 0), (3, 3)])[0]
    yield "hub_in_one_window", synth.graph_from_edges(
        700, [(u, v) for u in range(0, 700, 7) for v in range(600, 700)])[0]


@pytest.mark.parametrize("mode", MODES)
def test_special_graphs(ctx, mode):
    for name, g in special_graphs():
        dg, od, t = upload(g)
        for k in (0, 3, 20):
            ref = reference(g, t, k)
            got = ctx.pagerank(dg, od, k, mode=mode).cpu().numpy()
            assert oracle.pagerank_check(ref, got, bound(t, k, mode)) == (0, -1), (name, k)


def test_invalid_arguments(ctx, c1_pr):
    g, dg, od, t, refs = c1_pr
    for kw in (dict(iterations=-1), dict(damping=1.5), dict(damping=float("nan"))):
        args = dict(iterations=3, damping=0.85)
        args.update(kw)
        with pytest.raises(wc.WcError):
            ctx.pagerank(dg, od, args["iterations"], damping=args["damping"])
    with pytest.raises(wc.WcError):
        ctx.pagerank(dg, od, 3, mode=9)
    for driver in (1, 2, 3):
        with pytest.raises(wc.WcError):
            ctx.pagerank(dg, od, 3, mode="grid", tune=wc.make_tune(driver=driver))


def test_stats(ctx, c1_pr):
    g, dg, od, t, refs = c1_pr
    _, st = ctx.pagerank(dg, od, 10, mode="grid", stats=True)
    assert st["rounds"] == 10 and st["edges_processed"] == 10 * t.row_ptr[-1]
    assert 0 < st["edges_buffered"] < st["edges_processed"]


@pytest.fixture(scope="module")
def c2_pr():
    say("generating scale-22 graph for PageRank")
    g = synth.rmat_csr(22, 1 << 26)
    dg, od, t = upload(g)
    say("oracle PageRank at scale 22 (1 and 10 sweeps)")
    return g, dg, od, t, {k: reference(g, t, k) for k in (1, 10)}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("iters", [1, 10])
def test_scale22(ctx, c2_pr, mode, iters):
    """One sweep shows the first sums' rounding undamped (the hub's 159,737
    in-edges); ten sweeps the accumulated error.  Both against the bound derived
    for the mode."""
    g, dg, od, t, refs = c2_pr
    say(f"pagerank scale 22 mode={mode} iterations={iters}")
    got = ctx.pagerank(dg, od, iters, mode=mode).cpu().numpy()
    rtol = bound(t, iters, mode)
    assert rtol < (1e-5 if iters == 1 else 1e-4)
    assert oracle.pagerank_check(refs[iters], got, rtol) == (0, -1)
