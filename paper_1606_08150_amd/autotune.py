"""Autotuner for batched SSSP: per size bucket, the consolidation granularity,
threshold and items per lane (the Table I clauses consldt, threads/blocks and
the buffer estimate of Sec. IV.E), and one workgroup shape for the batch.

The paper compares its KC_X defaults with an exhaustive search of the kernel
configuration space (Sec. V.B); here the same comparison is made for the
batch: `heuristic_config` is the library default, and `tune` searches the
configurations one size bucket at a time (largest instances first), timing
every candidate of that bucket on the whole batch as it runs (graph-captured
rounds) with the other buckets at their best so far, then the workgroup
shape.  The search starts from the best of the default and the tables that
put every bucket at the wave or the block level (the buckets share one
launch, whose shape depends on the levels present, so a table can pay off
only when all buckets change together).  The library default is one of the
candidates at every step, so the table found is never slower than the
default on the batch it was tuned on (up to timing noise).  Tables are plain
JSON.
"""
from __future__ import annotations

import json
import math

# vertex-count buckets by floor(log2 n): [10,12), [12,14), [14,16), [16,19)
BUCKET_EDGES = (12, 14, 16)
MODES = ("flat", "wave", "block", "grid")
THRESHOLDS = (2, 4, 8, 16, 32, 64, 128)
ITEMS_PER_LANE = (1, 2, 4, 8, 16)       # grid level: chunk sizes (64 x items per lane)
BLOCKS = (128, 256, 512, 1024)


def bucket_of(n: int) -> int:
    lg = int(math.floor(math.log2(max(1, n))))
    b = 0
    for edge in BUCKET_EDGES:
        if lg >= edge:
            b += 1
    return b


def candidates():
    """Every (mode, threshold, items per lane) of the search: flat once (no
    threshold), wave and block per threshold, grid per threshold and chunk size
    (the batch's wave and block levels keep every buffered item in the group,
    so items per lane shapes only grid-level chunks)."""
    out = [{"mode": "flat", "threshold": 0, "items_per_lane": 0}]
    for mode in MODES[1:]:
        for thr in THRESHOLDS:
            for ipl in (ITEMS_PER_LANE if mode == "grid" else (0,)):
                out.append({"mode": mode, "threshold": thr, "items_per_lane": ipl})
    return out


def heuristic_config() -> dict:
    """The library's own choice (grid level, KC_1 drain, default threshold)."""
    return {"mode": "grid", "threshold": 0, "items_per_lane": 0}


def per_instance(table: dict, sizes) -> tuple[list, list]:
    """(modes, tune dicts) for instances of the given vertex counts; a
    workgroup shape of 0 (or none) is the library default."""
    from . import wc
    modes, tunes = [], []
    block = int(table.get("block_threads", 0))
    for n in sizes:
        cfg = table["buckets"].get(str(bucket_of(n)), heuristic_config())
        modes.append(cfg["mode"])
        tunes.append(wc.make_tune(threshold=cfg["threshold"], items_per_lane=cfg["items_per_lane"],
                                  block_threads=block))
    return modes, tunes


def save(table: dict, path: str):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


def _time_batch(ctx, graphs, weights, sources, modes, tunes, reps):
    """Median ms of the batch as it runs: the rounds it needs (plus two)
    captured into a graph, captured once untimed, then `reps` timed replays."""
    import torch
    stream = torch.cuda.current_stream()
    outs, st = ctx.sssp_batch(graphs, weights, sources, modes=modes, tunes=tunes, stats=True)
    rounds = st["rounds"] + 2
    ctx.sssp_batch(graphs, weights, sources, modes=modes, tunes=tunes, outs=outs, graph_rounds=rounds)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.sssp_batch(graphs, weights, sources, modes=modes, tunes=tunes, outs=outs, graph_rounds=rounds)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return sorted(times)[len(times) // 2]


def tune(ctx, graphs, weights, sources, reps: int = 2) -> dict:
    """Coordinate search over the buckets present (largest first), then over
    the workgroup shapes, every trial timed on the whole batch; returns the
    table with the default's time, each bucket's trials and the final time."""
    sizes = [g.n for g in graphs]
    present = sorted({bucket_of(n) for n in sizes}, reverse=True)
    table = {"buckets": {str(b): heuristic_config() for b in present}, "timings_ms": {}, "block_threads": 0}

    def run(tbl):
        modes, tunes = per_instance(tbl, sizes)
        return _time_batch(ctx, graphs, weights, sources, modes, tunes, reps)

    best_ms = heur_ms = run(table)
    uniform = {}
    for mode in ("wave", "block"):
        start = {"buckets": {str(b): {"mode": mode, "threshold": 0, "items_per_lane": 0} for b in present},
                 "block_threads": 0}
        ms = run(start)
        uniform[mode] = round(ms, 4)
        if ms < best_ms:
            best_ms = ms
            table["buckets"] = dict(start["buckets"])
    for b in present:
        trials = []
        for cfg in candidates():
            trial = {"buckets": dict(table["buckets"], **{str(b): cfg}), "block_threads": 0}
            trials.append((run(trial), cfg))
        ms, cfg = min(trials, key=lambda r: r[0])
        if ms < best_ms:
            best_ms = ms
            table["buckets"][str(b)] = cfg
        table["timings_ms"][str(b)] = {"instances": sum(1 for n in sizes if bucket_of(n) == b),
                                       "all": [[round(t, 4), c] for t, c in trials]}
    for block in BLOCKS:
        ms = run(dict(table, block_threads=block))
        if ms < best_ms:
            best_ms = ms
            table["block_threads"] = block
    table["timings_ms"]["heuristic"] = round(heur_ms, 4)
    table["timings_ms"]["uniform"] = uniform
    table["timings_ms"]["whole_batch_tuned"] = round(best_ms, 4)
    return table
