"""Host-side logic of the batch autotuner (no GPU)."""
import os
import tempfile

from paper_1606_08150_amd import autotune


def test_buckets_follow_log2_size():
    assert [autotune.bucket_of(n) for n in (1024, 4095, 4096, 16383, 16384, 65535, 65536, 262144)] == \
        [0, 0, 1, 1, 2, 2, 3, 3]


def test_candidates_cover_the_search_space_once():
    c = autotune.candidates()
    assert {x["mode"] for x in c} == {"flat", "wave", "block", "grid"}
    assert len([x for x in c if x["mode"] == "flat"]) == 1
    assert len([x for x in c if x["mode"] == "grid"]) == len(autotune.THRESHOLDS) * len(autotune.ITEMS_PER_LANE)
    for mode in ("wave", "block"):
        assert len([x for x in c if x["mode"] == mode]) == len(autotune.THRESHOLDS)
    keys = [(x["mode"], x["threshold"], x["items_per_lane"]) for x in c]
    assert len(keys) == len(set(keys))


def test_table_roundtrip_and_per_instance_lookup():
    table = {"buckets": {"0": {"mode": "wave", "threshold": 8, "items_per_lane": 4},
                         "3": {"mode": "grid", "threshold": 32, "items_per_lane": 8}},
             "block_threads": 512, "timings_ms": {}}
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "t.json")
        autotune.save(table, p)
        t2 = autotune.load(p)
    assert t2 == table
    modes, tunes = autotune.per_instance(t2, [2000, 300000, 20000])
    assert modes == ["wave", "grid", "grid"]
    assert [t.threshold for t in tunes] == [8, 32, 0]  # bucket 2 absent: the heuristic default
    assert {t.block_threads for t in tunes} == {512}


class _G:
    def __init__(self, n):
        self.n = n


def test_coordinate_search_finds_the_best_separable_table(monkeypatch):
    """With a batch time that is a sum of per-instance costs, the search by
    buckets (then workgroup shapes) lands on the cheapest configuration of every
    bucket, and never reports a table slower than the default."""
    best = {0: ("block", 4, 0), 1: ("grid", 16, 2), 3: ("wave", 8, 0)}

    def cost(n, tune, mode):
        b = autotune.bucket_of(n)
        want = best.get(b, ("grid", 0, 0))
        c = 1.0 if (mode, tune.threshold, tune.items_per_lane) == want else 2.0
        return c + (0.0 if tune.block_threads in (0, 512) else 0.5)

    def fake_time(ctx, graphs, weights, sources, modes, tunes, reps):
        return sum(cost(g.n, t, m) for g, t, m in zip(graphs, tunes, modes))

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    graphs = [_G(n) for n in (1500, 2000, 5000, 9000, 70000, 200000)]
    table = autotune.tune(None, graphs, [None] * len(graphs), [0] * len(graphs), reps=1)
    for b, (mode, thr, ipl) in best.items():
        assert table["buckets"][str(b)] == {"mode": mode, "threshold": thr, "items_per_lane": ipl}
    assert "2" not in table["buckets"]  # no instance in that bucket: nothing searched
    assert table["block_threads"] == 0
    assert table["timings_ms"]["whole_batch_tuned"] == 6.0 < table["timings_ms"]["heuristic"]


def test_uniform_start_reaches_a_joint_optimum(monkeypatch):
    """Buckets that only pay off together (block level is cheap when every
    instance runs at block level, dear otherwise): one bucket at a time from
    the default cannot leave it, the uniform start can, and the search keeps
    the joint table."""
    def fake_time(ctx, graphs, weights, sources, modes, tunes, reps):
        all_block = all(m == "block" for m in modes)
        return sum((1.5 if all_block else 2.5) if m == "block" else 2.0 for m in modes)

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    graphs = [_G(n) for n in (1500, 5000, 20000, 200000)]
    table = autotune.tune(None, graphs, [None] * len(graphs), [0] * len(graphs), reps=1)
    assert {c["mode"] for c in table["buckets"].values()} == {"block"}
    assert table["timings_ms"]["heuristic"] == 8.0
    assert table["timings_ms"]["uniform"] == {"wave": 8.0, "block": 6.0}
    assert table["timings_ms"]["whole_batch_tuned"] == 6.0
