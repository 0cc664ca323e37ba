"""Benchmark: workload consolidation on the scale-22 R-MAT graph, one MI355X.

Workload (the headline configuration): R-MAT with 2^22 vertices and 2^26
directed edges (a, b, c, d = 0.57, 0.19, 0.19, 0.05), int32 CSR, uint32 weights
uniform in [1, 100], fp32 values and x uniform in [-1, 1), all seeded and
synthetic.  One step = one SSSP from vertex 0 plus one SpMV, both in the
headline consolidation mode (grid by default), inputs resident in HBM.

Printed as one JSON line:
  value        SSSP GTEPS = edges out of reached vertices / SSSP time, over the
               timed steps (the SpMV's rate is reported beside it)
  modes        flat / wave / block / grid side by side (SSSP GTEPS, SpMV GB/s)
  roofline     the step's dominant kernel: algorithmic bytes per launch divided
               by its event-measured average launch duration, against 8 TB/s
  cpu_baseline the oracle (binary-heap Dijkstra) on this host, GTEPS
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INF = 0xFFFFFFFF


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--mode", default="grid", choices=["flat", "wave", "block", "grid"])
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--edge-factor", type=int, default=16)
    p.add_argument("--no-modes", action="store_true", help="skip the flat/wave/block/grid side-by-side table")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-reps", type=int, default=5)
    return p.parse_args()


def algorithmic_bytes(kernel: str, info: dict) -> tuple[float, str] | None:
    """Algorithmic bytes a launch of `kernel` must move (read once), from the
    per-unit figures: SpMV 12 B per nonzero (col, val, x gather) + 8 B per row
    (row_ptr, y); SSSP 16 B per edge (col, w, dist read-modify-write) + 20 B per
    frontier vertex (row_ptr pair, dist, frontier in/out)."""
    if kernel == "spmv_drain":
        return 12.0 * info["nnz_heavy"] + 4.0 * info["rows_heavy"], "nnz in buffered rows x 12 B + rows x 4 B"
    if kernel.startswith("spmv_parent"):
        return (12.0 * info["nnz_light"] + 8.0 * info["n"],
                "nnz in inline rows x 12 B + rows x 8 B (row_ptr, y)")
    if kernel in ("sssp_drain",) or kernel.startswith("sssp_round"):
        return None
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1606_08150_amd import wc

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t0 = time.time()
    scale, m = args.scale, (1 << args.scale) * args.edge_factor
    g = synth.rmat_csr(scale, m)
    w = synth.weights(g.m)
    val, x = synth.values(g.m), synth.vector_x(g.n)
    print(f"[bench] inputs generated in {time.time() - t0:.1f}s (n={g.n}, m={g.m})", file=sys.stderr, flush=True)

    ctx = wc.Context(0)
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = torch.from_numpy(w.view(np.int32)).cuda()
    dval, dx = torch.from_numpy(val).cuda(), torch.from_numpy(x).cuda()
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    deg = torch.from_numpy(np.diff(g.row_ptr).astype(np.int64)).cuda()
    stream = torch.cuda.current_stream()

    def sssp(mode):
        ctx.sssp(dg, dw, 0, mode=mode, out=dist)

    def spmv(mode):
        ctx.spmv(dg, dval, dx, mode=mode, out=y)

    # reached edges (GTEPS numerator) from the GPU result: out-edges of vertices with finite distance
    sssp(args.mode)
    torch.cuda.synchronize()
    reached_mask = dist != -1  # INF as int32
    m_reached = int(deg[reached_mask].sum().item())
    n_reached = int(reached_mask.sum().item())

    # ---- timed region: K steps of (SSSP + SpMV), per-kernel events on the launch stream
    for _ in range(args.warmup):
        sssp(args.mode)
        spmv(args.mode)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        a, b, c = ev[k]
        a.record(stream)
        sssp(args.mode)
        b.record(stream)
        spmv(args.mode)
        c.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    sssp_ms = [e[0].elapsed_time(e[1]) for e in ev]
    spmv_ms = [e[1].elapsed_time(e[2]) for e in ev]
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)
    ms_per_step = wall * 1e3 / args.steps
    sssp_avg = float(np.mean(sssp_ms))
    spmv_avg = float(np.mean(spmv_ms))
    gteps = m_reached / (sssp_avg * 1e-3) / 1e9
    spmv_bytes = 12.0 * g.m + 8.0 * g.n
    spmv_gbs = spmv_bytes / (spmv_avg * 1e-3) / 1e9

    # ---- roofline of the dominant kernel
    lens = np.diff(g.row_ptr).astype(np.int64)
    thr = wc.default_tune("spmv", args.mode, 1)["threshold"]
    heavy = lens > thr
    info = dict(n=g.n, nnz_heavy=int(lens[heavy].sum()), rows_heavy=int(heavy.sum()),
                nnz_light=int(lens[~heavy].sum()))
    dominant = max(ktimes.items(), key=lambda kv: kv[1][1])
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 4), "avg_ms": round(v[1] / v[0], 5)}
               for k, v in sorted(ktimes.items(), key=lambda kv: -kv[1][1])}
    roofline = None
    # the largest kernel with an algorithmic-byte model
    for name, (launches, total, _) in sorted(ktimes.items(), key=lambda kv: -kv[1][1]):
        ab = algorithmic_bytes(name, info)
        if ab is None:
            continue
        bytes_per_launch, what = ab
        avg_s = total / launches * 1e-3
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "bytes_per_launch": bytes_per_launch, "bytes_model": what,
                    "avg_launch_ms": round(total / launches, 5), "dominant_kernel": dominant[0],
                    "is_dominant": name == dominant[0]}
        break

    # ---- flat / wave / block / grid side by side (1 timed run each after 1 warm-up)
    modes = {}
    if not args.no_modes:
        for mode in ("flat", "wave", "block", "grid"):
            res = {}
            for prob, fn in (("sssp", sssp), ("spmv", spmv)):
                fn(mode)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 3
                a.record(stream)
                for _ in range(reps):
                    fn(mode)
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / reps
                res[prob + "_ms"] = round(ms, 3)
            res["sssp_gteps"] = round(m_reached / (res["sssp_ms"] * 1e-3) / 1e9, 3)
            res["spmv_gbs"] = round(spmv_bytes / (res["spmv_ms"] * 1e-3) / 1e9, 1)
            modes[mode] = res
            print(f"[bench] mode {mode}: {res}", file=sys.stderr, flush=True)

    # ---- CPU baseline: the oracle's Dijkstra on the same graph, this host
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps = max(1, args.cpu_reps)
        t1 = time.perf_counter()
        for _ in range(reps):
            ref = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
        dt = (time.perf_counter() - t1) / reps
        cpu = {"value": round(oracle.sssp_reached_edges(g.row_ptr, ref) / dt / 1e9, 5), "unit": "GTEPS",
               "cores": 1, "kind": "oracle",
               "sample": f"binary-heap Dijkstra from vertex 0 on the full scale-{scale} graph, {reps} runs "
                         f"(mean {dt:.2f} s each)"}

    out = {
        "metric": "GTEPS (SSSP) + GB/s vs HBM peak, consolidated vs flat; p99 batched latency",
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (SSSP) / f32 (SpMV)",
        "data": "synthetic (seeded R-MAT, no dataset)",
        "config": {"workload": f"R-MAT scale {scale}, {m} edges, SSSP from vertex 0 + SpMV, mode {args.mode}",
                   "n": g.n, "m": g.m, "mode": args.mode, "reached_vertices": n_reached,
                   "reached_edges": m_reached},
        "sssp_ms": round(sssp_avg, 4),
        "spmv_ms": round(spmv_avg, 4),
        "spmv_gbs": round(spmv_gbs, 1),
        "spmv_frac_hbm": round(spmv_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels": kernels,
        "modes": modes,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
