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
