"""GPU parity of wc_sssp_batch: every instance bit-exact against the oracle,
mixed per-instance modes, graph capture and replays (with eager work between
replays), rounds beyond the captured graph, edge-case instances, autotuner."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, say, u32_to_dev
from paper_1606_08150_amd import autotune, wc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_batch():
    inst = synth.batch_instances(24, lo_log2=6, hi_log2=13, seed=41)
    # edge cases: a single vertex, an isolated source, a chain
    inst.append(synth.graph_from_edges(1, [], []))
    inst.append(synth.graph_from_edges(50, [(1, 2), (2, 3)], [3, 4]))
    inst.append(synth.graph_from_edges(300, [(i, i + 1) for i in range(299)], [1 + i % 9 for i in range(299)]))
    graphs = [wc.DeviceCSR.from_host(g.row_ptr, g.col) for g, _ in inst]
    weights = [u32_to_dev(np.asarray(w, np.uint32)) for _, w in inst]
    srcs = [0] * len(inst)
    refs = [oracle.sssp_dijkstra(g.row_ptr, g.col, np.asarray(w, np.uint32), 0) for g, w in inst]
    return graphs, weights, srcs, refs


def check(outs, refs):
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(dev_to_u32(o), r), f"instance {i}"


@pytest.mark.parametrize("mode", ["flat", "wave", "block", "grid"])
def test_uniform_mode(ctx, small_batch, mode):
    graphs, weights, srcs, refs = small_batch
    say(f"batch mode={mode}")
    outs = ctx.sssp_batch(graphs, weights, srcs, modes=[mode] * len(graphs))
    torch.cuda.synchronize()
    check(outs, refs)


def test_mixed_modes_and_tunes(ctx, small_batch):
    graphs, weights, srcs, refs = small_batch
    ms = ["flat", "wave", "block", "grid"]
    modes = [ms[i % 4] for i in range(len(graphs))]
    tunes = [wc.make_tune(threshold=1 + 7 * (i % 5), items_per_lane=1 << (i % 4)) for i in range(len(graphs))]
    for block in (64, 256, 1024):
        for t in tunes:
            t.block_threads = block
        say(f"batch mixed block={block}")
        outs, st = ctx.sssp_batch(graphs, weights, srcs, modes=modes, tunes=tunes, stats=True)
        torch.cuda.synchronize()
        check(outs, refs)
        assert st["rounds"] >= 1 and st["items_buffered"] > 0


def test_graph_capture_and_replays(ctx, small_batch):
    graphs, weights, srcs, refs = small_batch
    modes = ["grid"] * len(graphs)
    # fewer captured rounds than needed (continues with ordinary rounds), about
    # enough, and more than enough; each replayed several times with eager work
    # (another SSSP, a synchronization) between the replays
    g0 = graphs[5]
    eager_ref = refs[5]
    for rounds in (2, 12, 40):
        for rep in range(4):
            say(f"batch graph_rounds={rounds} replay={rep}")
            outs = ctx.sssp_batch(graphs, weights, srcs, modes=modes, graph_rounds=rounds)
            torch.cuda.synchronize()
            check(outs, refs)
            d = ctx.sssp(g0, weights[5], 0, mode="block")
            torch.cuda.synchronize()
            assert np.array_equal(dev_to_u32(d), eager_ref)


def test_bad_arguments(ctx, small_batch):
    graphs, weights, srcs, refs = small_batch
    with pytest.raises(wc.WcError):
        ctx.sssp_batch(graphs[:3], weights[:3], [0, 0, 10 ** 9])
    t = [wc.make_tune(block_threads=256), wc.make_tune(block_threads=512)]
    with pytest.raises(wc.WcError):
        ctx.sssp_batch(graphs[:2], weights[:2], [0, 0], tunes=t)
    assert ctx.sssp_batch([], [], []) == []


def test_autotuner_table_gives_exact_results(ctx, small_batch):
    graphs, weights, srcs, refs = small_batch
    say("autotune")
    table = autotune.tune(ctx, graphs, weights, srcs, reps=1)
    assert set(table["buckets"]) and table["block_threads"] in (0,) + autotune.BLOCKS
    # the default is a candidate at every step of the search
    assert table["timings_ms"]["whole_batch_tuned"] <= table["timings_ms"]["heuristic"]
    modes, tunes = autotune.per_instance(table, [g.n for g in graphs])
    outs = ctx.sssp_batch(graphs, weights, srcs, modes=modes, tunes=tunes, graph_rounds=16)
    torch.cuda.synchronize()
    check(outs, refs)


@pytest.fixture(scope="module")
def full_batch():
    """The 512-instance batch at its full size (25.2M vertices, 403M edges)."""
    say("generating the 512-instance batch")
    inst = synth.batch_instances(512)
    graphs = [wc.DeviceCSR.from_host(g.row_ptr, g.col) for g, _ in inst]
    weights = [u32_to_dev(np.asarray(w, np.uint32)) for _, w in inst]
    yield inst, graphs, weights
    del graphs, weights
    torch.cuda.empty_cache()


def test_full_batch_certified_and_sampled_exact(ctx, full_batch):
    """Every instance passes the shortest-path certificate; a seeded sample
    (with the smallest and the largest instance) equals the oracle's Dijkstra."""
    inst, graphs, weights = full_batch
    srcs = [0] * len(inst)
    for rounds in (0, 16):
        say(f"full batch graph_rounds={rounds}")
        outs = ctx.sssp_batch(graphs, weights, srcs, modes=["grid"] * len(inst), graph_rounds=rounds)
        torch.cuda.synchronize()
        got = [dev_to_u32(o) for o in outs]
        for i, ((g, w), d) in enumerate(zip(inst, got)):
            assert oracle.sssp_certify(g.row_ptr, g.col, np.asarray(w, np.uint32), 0, d) == (0, -1), i
    sizes = np.array([g.n for g, _ in inst])
    rng = np.random.default_rng(12)
    sample = {int(sizes.argmin()), int(sizes.argmax())} | set(rng.choice(len(inst), 14, replace=False).tolist())
    for i in sorted(sample):
        g, w = inst[i]
        assert np.array_equal(got[i], oracle.sssp_dijkstra(g.row_ptr, g.col, np.asarray(w, np.uint32), 0)), i
