"""Host-side logic of the batch autotuner (no GPU)."""
import os
import tempfile

from paper_1606_08150_amd import autotune


def test_buckets_follow_log2_size():
    assert [autotune.bucket_of(n) for n in (1024, 4095, 4096, 16383, 16384, 65535, 65536, 262144)] == \
        [0, 0, 1, 1, 2, 2, 3, 3]


def test_candidates_cover_every_mode_once_per_threshold():
    c = autotune.candidates()
    assert {x["mode"] for x in c} == {"wave", "block", "grid"}
    assert len([x for x in c if x["mode"] == "grid"]) == len(autotune.THRESHOLDS) * len(autotune.ITEMS_PER_LANE)
    assert len([x for x in c if x["mode"] == "wave"]) == len(autotune.THRESHOLDS)


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
