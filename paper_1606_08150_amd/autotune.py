"""Autotuner for batched SSSP: per size bucket, the consolidation granularity,
threshold and items per lane (the Table I clauses consldt, threads/blocks and
the buffer estimate of Sec. IV.E), and one workgroup shape for the batch.

The paper compares its KC_X defaults with an exhaustive search of the kernel
configuration space (Sec. V.B); here the same comparison is made per size
bucket: `heuristic_config` is the library default, `tune` times every candidate
on a sample of each bucket's instances through wc_sssp_batch and keeps the
fastest.  Tables are plain JSON.
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
    """(modes, tune dicts) for instances of the given vertex counts."""
    from . import wc
    modes, tunes = [], []
    block = int(table.get("block_threads", 256))
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
    import torch
    stream = torch.cuda.current_stream()
    outs = ctx.sssp_batch(graphs, weights, sources, modes=modes, tunes=tunes)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        ctx.sssp_batch(graphs, weights, sources, modes=modes, tunes=tunes, outs=outs)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(ctx, graphs, weights, sources, sample: int = 32, reps: int = 3) -> dict:
    """Times every candidate per bucket (on up to `sample` instances of that
    bucket) and every workgroup shape on the whole batch; returns the table
    with the measured times of the heuristic and of the chosen configuration."""
    from . import wc
    by_bucket: dict[int, list[int]] = {}
    for i, g in enumerate(graphs):
        by_bucket.setdefault(bucket_of(g.n), []).append(i)
    table = {"buckets": {}, "timings_ms": {}, "block_threads": 256}
    for b, idx in sorted(by_bucket.items()):
        idx = idx[:sample]
        gs, ws, ss = [graphs[i] for i in idx], [weights[i] for i in idx], [sources[i] for i in idx]
        results = []
        for cfg in [heuristic_config()] + candidates():
            t = wc.make_tune(threshold=cfg["threshold"], items_per_lane=cfg["items_per_lane"])
            ms = _time_batch(ctx, gs, ws, ss, [cfg["mode"]] * len(gs), [t] * len(gs), reps)
            results.append((ms, cfg))
        heur_ms = results[0][0]
        best_ms, best = min(results, key=lambda r: r[0])
        table["buckets"][str(b)] = best
        table["timings_ms"][str(b)] = {"instances": len(idx), "heuristic": round(heur_ms, 4),
                                       "tuned": round(best_ms, 4),
                                       "all": [[round(ms, 4), cfg] for ms, cfg in results]}
    sizes = [g.n for g in graphs]
    best_block, best_ms = 256, None
    for block in BLOCKS:
        table["block_threads"] = block
        modes, tunes = per_instance(table, sizes)
        ms = _time_batch(ctx, graphs, weights, sources, modes, tunes, reps)
        if best_ms is None or ms < best_ms:
            best_block, best_ms = block, ms
    table["block_threads"] = best_block
    table["timings_ms"]["whole_batch_tuned"] = round(best_ms, 4)
    return table
