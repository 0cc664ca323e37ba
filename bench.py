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
               (and against the attainable rate of a plain 1 GiB device copy)
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
    p.add_argument("--cpu-reps", type=int, default=8)
    p.add_argument("--no-batch", action="store_true", help="skip the 512-instance batched SSSP section")
    p.add_argument("--batch-count", type=int, default=512)
    p.add_argument("--batch-reps", type=int, default=10)
    p.add_argument("--no-trees", action="store_true", help="skip the tree descendants / heights section")
    p.add_argument("--no-serve", action="store_true", help="skip the continuous-batching serving section")
    p.add_argument("--serve-requests", type=int, default=10000, help="requests per arrival rate")
    p.add_argument("--no-gather-ceiling", action="store_true", help="skip the bare-gather reference timing")
    p.add_argument("--no-spmv-hot", action="store_true", help="skip the hot-column SpMV layout timings")
    p.add_argument("--no-cold", action="store_true", help="skip the cold-cache (L2 and MALL flushed) timings")
    p.add_argument("--no-pagerank", action="store_true", help="skip the PageRank section")
    p.add_argument("--no-coloring", action="store_true", help="skip the graph coloring section")
    p.add_argument("--no-ablation", action="store_true", help="skip the basic dynamic parallelism comparison")
    p.add_argument("--no-config-search", action="store_true",
                   help="skip the comparison of the default configuration with exhaustive search")
    p.add_argument("--serve-rates", default="1000,2000,5000,10000,20000")
    p.add_argument("--serve-workers", type=int, default=4)
    p.add_argument("--serve-sssp-mode", default="grid", choices=["flat", "wave", "block", "grid"],
                   help="consolidation level of the serving section's batched SSSP requests")
    p.add_argument("--counter-run", default=None, choices=["flat", "wave", "block", "grid"],
                   help="only run SSSP, SpMV and tree descendants in this mode, 3 calls each (for rocprofv3 "
                        "counter passes per mode), then exit")
    p.add_argument("--calibrate-copy-mb", type=int, default=0,
                   help="first run a plain device-to-device copy of this many MiB three times (a known-size "
                        "kernel for scaling hardware byte counters)")
    p.add_argument("--jsonl", default=None, help="also append the result line to this JSONL file")
    return p.parse_args()


def algorithmic_bytes(kernel: str, info: dict, launches: int) -> tuple[float, str] | None:
    """Algorithmic bytes per launch of `kernel` (each datum read or written once),
    from the per-unit figures: SpMV 12 B per nonzero (col, val, x gather) + 8 B
    per row (row_ptr, y); SSSP 16 B per reachable edge (col 4, w 4, dist[v] read
    and write 8) + 20 B per reached vertex (row_ptr 8, dist[u] 4, frontier in and
    out 8), each edge and vertex counted once however often the schedule relaxes
    it (re-relaxations are overhead, not useful bytes).  The SSSP drain handles
    the reached vertices above the grid threshold, the parent the others.  For
    kernels launched once per round the units are the per-call totals spread over
    that call's launches (empty trailing rounds included)."""
    if kernel == "spmv_drain":
        return 12.0 * info["nnz_heavy"] + 4.0 * info["rows_heavy"], "12 B x nonzeros of buffered rows + 4 B x rows"
    if kernel == "spmv_parent_grid":
        return (12.0 * info["nnz_light"] + 8.0 * info["n"],
                "12 B x nonzeros of inline rows + 8 B x rows (row_ptr, y)")
    if kernel == "sssp_drain":
        per_call = 16.0 * info["reached_edges_heavy"] + 20.0 * info["reached_heavy"]
        return (per_call * info["sssp_calls"] / launches,
                "16 B x reachable edges of reached vertices above the threshold (col, w, dist read + write) "
                "+ 20 B x those vertices (row_ptr, dist, frontier in + out)")
    if kernel.startswith("sssp_round"):
        per_call = 16.0 * info["reached_edges_light"] + 20.0 * info["reached_light"]
        return (per_call * info["sssp_calls"] / launches,
                "16 B x reachable edges of reached vertices up to the threshold + 20 B x those vertices")
    return None


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def counter_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>_<workload>_pmc.json (FETCH_SIZE and WRITE_SIZE scaled by the
    copy calibration), or None when absent or taken on different kernel sources."""
    symbol = {"sssp_round_grid": "sssp_round_grid2"}.get(kernel, kernel)  # counter files use the kernel symbol
    path = os.path.join(ROOT, "profiles", f"{symbol}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1606_08150_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def _short_kernel(name: str) -> str:
    import re
    m = re.search(r"(\w+)(<[^()]*>)?\(", name.replace("(anonymous namespace)", "anon"))
    return m.group(1) if m else name


def summarize_kernel_stats(stats_csv, workload, command, out_name):
    """profiles/<out_name>.md from a rocprofv3 --kernel-trace --stats csv."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel statistics: {workload}", "", "Command:", "", "```", command, "```", "",
             "| kernel (symbol) | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {_short_kernel(r['Name'])} `{r['Name'][:70]}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['Percentage']):.2f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def static_resources(kernels):
    """{kernel: (VGPRs, scratch B/lane, waves per SIMD, LDS B/block)} of the 512-thread
    instantiations the timed path runs, from hipcc's kernel-resource-usage remarks on the sources."""
    import re
    import subprocess
    csrc = os.path.join(ROOT, "paper_1606_08150_amd", "csrc")
    out = {}
    for src in ("wc_sssp.hip", "wc_spmv.hip"):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-c", os.path.join(csrc, src),
               "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]
        text = subprocess.run(cmd, capture_output=True, text=True).stderr
        cur = None
        for line in text.splitlines():
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                # the instantiation the timed path runs: every bool parameter
                # (stamps, stats, hot columns) false
                cur = next((k for k in kernels if f"{len(k)}{k}ILi512E" in name and "Lb1E" not in name), None)
                if cur:
                    out[cur] = {}
                continue
            if cur is None:
                continue
            for key, pat in (("vgprs", r"VGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                             ("waves", r"Occupancy \[waves/SIMD\]: (\d+)"), ("lds", r"LDS Size \[bytes/block\]: (\d+)")):
                m = re.search(pat, line)
                if m:
                    out[cur][key] = int(m.group(1))
    return out


def summarize_counters(sq_dir, tcc_dir, workload, command, out_name,
                       kernels=("sssp_drain", "sssp_round_grid2", "spmv_drain", "spmv_parent_grid"),
                       with_static=True, cyc_dir=None, cyc_command=None):
    """profiles/<out_name>.md: per-kernel wave, VALU, memory-instruction, L2 and
    atomic counters from two rocprofv3 --pmc runs (SQ_* + GRBM_GUI_ACTIVE, then
    TCC_*), summed over each kernel's dispatches, and the static resources
    (registers, scratch, occupancy, LDS) from hipcc's resource-usage remarks."""
    import csv
    tot = {}
    for d in (sq_dir, tcc_dir):
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                k = _short_kernel(r["Kernel_Name"])
                if k not in kernels:
                    continue
                ent = tot.setdefault(k, {"dispatches": set(), "wg": int(r["Workgroup_Size"])})
                ent["dispatches"].add((d, r["Dispatch_Id"]))
                ent[r["Counter_Name"]] = ent.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# Counters: {workload}", "", "Commands (two passes):", "", "```", command, "```", "",
             "Sums over every dispatch of the kernel in the run. Ratios of SQ sums are relative measures "
             "(the SQ counters are accumulated over all shader engines).", "",
             "| kernel | dispatches | workgroup | waves | VALU insts / wave | VMEM reads / wave | wave-cycles / wave "
             "| VALU-active / wave-cycles | waiting / wave-cycles | L2 hit rate | L2 atomics / dispatch "
             "| EA atomics / dispatch |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]

    def per(x, y):
        return f"{x / y:.2f}" if y else "-"
    for k in kernels:
        if k not in tot:
            continue
        e = tot[k]
        nd = len({i for (d, i) in e["dispatches"] if d == sq_dir}) or 1
        ntcc = len({i for (d, i) in e["dispatches"] if d == tcc_dir}) or 1
        waves, wcyc = e.get("SQ_WAVES", 0.0), e.get("SQ_WAVE_CYCLES", 0.0)
        hit, miss = e.get("TCC_HIT_sum", 0.0), e.get("TCC_MISS_sum", 0.0)
        lines.append(f"| {k} | {nd} | {e['wg']} | {waves:.0f} | {per(e.get('SQ_INSTS_VALU', 0.0), waves)} | "
                     f"{per(e.get('SQ_INSTS_VMEM_RD', 0.0), waves)} | {per(wcyc, waves)} | "
                     f"{per(e.get('SQ_ACTIVE_INST_VALU', 0.0), wcyc)} | {per(e.get('SQ_WAIT_INST_ANY', 0.0), wcyc)} | "
                     f"{per(hit, hit + miss)} | {e.get('TCC_ATOMIC_sum', 0.0) / ntcc:.0f} | "
                     f"{e.get('TCC_EA0_ATOMIC_sum', 0.0) / ntcc:.0f} |")
    if cyc_dir:
        cyc = {}
        with open(os.path.join(cyc_dir, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                k = _short_kernel(r["Kernel_Name"])
                if k in kernels:
                    cyc.setdefault(k, {})
                    cyc[k][r["Counter_Name"]] = cyc[k].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        cols = ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS")
        lines += ["", "Where the wave-cycles go (each counter over SQ_WAVE_CYCLES, same units):", "", "```",
                  cyc_command or "", "```", "",
                  "| kernel | " + " | ".join(c.replace("SQ_", "").lower() for c in cols) + " |",
                  "|---|" + "---|" * len(cols)]
        for k in kernels:
            if k in cyc and cyc[k].get("SQ_WAVE_CYCLES"):
                wcy = cyc[k]["SQ_WAVE_CYCLES"]
                lines.append(f"| {k} | " + " | ".join(f"{cyc[k].get(c, 0.0) / wcy:.3f}" for c in cols) + " |")
    res = static_resources(kernels) if with_static else {}
    if res:
        lines += ["", "Static resources of the 512-thread kernels (`hipcc --offload-arch=gfx950 -O3 -std=c++17 "
                  "-Xclang -target-feature -Xclang -packed-fp32-ops -c <wc_sssp.hip|wc_spmv.hip> "
                  "-Rpass-analysis=kernel-resource-usage`):", "",
                  "| kernel | VGPRs | scratch B/lane | waves/SIMD | LDS B/block |", "|---|---|---|---|---|"]
        for k in kernels:
            if k in res:
                r = res[k]
                lines.append(f"| {k} | {r.get('vgprs', '-')} | {r.get('scratch', '-')} | {r.get('waves', '-')} | "
                             f"{r.get('lds', '-')} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return tot


MODE_PROBLEMS = (("sssp", "sssp_"), ("spmv", "spmv_"), ("tree", "tree_"))


def summarize_mode_counters(runs, workload, command, out_name, fetch_scale=2.0):
    """profiles/<out_name>.md: the per-mode comparison of Figs. 8-10 (Sec. V.D)
    from rocprofv3 --pmc passes of `bench.py --counter-run MODE`, one process
    per mode and pass: `runs` maps mode -> output directories.  Per mode and
    problem, over that problem's kernels: VALU lane utilization (the analogue of
    warp execution efficiency: active lanes per VALU instruction / 64), mean
    waves per CU weighted by dispatch length (the occupancy analogue), and
    HBM-side bytes (FETCH_SIZE scaled by the copy calibration, plus WRITE_SIZE)
    per call."""
    import csv
    disp = {}
    for mode, dirs in runs.items():
        for d in dirs:
            with open(os.path.join(d, "run_counter_collection.csv")) as f:
                for r in csv.DictReader(f):
                    k = _short_kernel(r["Kernel_Name"])
                    prob = next((p for p, prefix in MODE_PROBLEMS if k.startswith(prefix)), None)
                    if prob is None:
                        continue
                    e = disp.setdefault((mode, prob, d, r["Dispatch_Id"]), {})
                    c = r["Counter_Name"]
                    e[c] = e.get(c, 0.0) + float(r["Counter_Value"])
    rows = {}
    for (mode, prob, _, _), e in disp.items():
        t = rows.setdefault((mode, prob), {"occ_w": 0.0, "gui": 0.0})
        for c, v in e.items():
            t[c] = t.get(c, 0.0) + v
        if "MeanOccupancyPerCU" in e and "GRBM_GUI_ACTIVE" in e:
            t["occ_w"] += e["MeanOccupancyPerCU"] * e["GRBM_GUI_ACTIVE"]
            t["gui"] += e["GRBM_GUI_ACTIVE"]
    lines = [f"# Counters per consolidation mode: {workload}", "",
             "Commands (one process per mode and counter pass):", "", "```", command, "```", "",
             "Over every kernel of the problem in the run (3 calls each). VALU lane utilization = "
             "SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU), the analogue of warp execution efficiency "
             "(Fig. 8); waves per CU = MeanOccupancyPerCU weighted by each dispatch's GRBM_GUI_ACTIVE cycles, "
             "the occupancy analogue (Fig. 9); HBM-side bytes = "
             f"{fetch_scale:g} x FETCH_SIZE + WRITE_SIZE (KiB counters, copy-calibrated) per call, the analogue "
             "of DRAM transactions (Fig. 10).", "",
             "| problem | mode | VALU insts per call | VALU lane utilization | waves per CU | HBM-side MB per call |",
             "|---|---|---|---|---|---|"]
    for prob, _ in MODE_PROBLEMS:
        for mode in ("flat", "wave", "block", "grid"):
            t = rows.get((mode, prob))
            if not t:
                continue
            act = t.get("SQ_ACTIVE_INST_VALU", 0.0)
            util = t.get("SQ_THREAD_CYCLES_VALU", 0.0) / (64.0 * act) if act else float("nan")
            occ = t["occ_w"] / t["gui"] if t["gui"] else float("nan")
            mb = (fetch_scale * t.get("FETCH_SIZE", 0.0) + t.get("WRITE_SIZE", 0.0)) * 1024 / 3 / 1e6
            lines.append(f"| {prob} | {mode} | {t.get('SQ_INSTS_VALU', 0.0) / 3:.3g} | {util:.3f} | {occ:.1f} | "
                         f"{mb:.1f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def summarize_profiles(fetch_dir, write_dir, copy_mb, workload, command):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; csv output) of
    `command` into profiles/<kernel>_<workload>_pmc.json files: KiB per dispatch
    scaled by what the same counters read for the calibration copy (a plain
    device copy of known size run first by the same command)."""
    import collections
    import csv

    def load(d, counter):
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] == counter:
                key = "calibration_copy" if "bitwise_not" in r["Kernel_Name"] else _short_kernel(r["Kernel_Name"])
                per[key].append(float(r["Counter_Value"]))
        return per

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copies = fetch["calibration_copy"]
    known = 3 * copy_mb * 1024.0 * 1024.0 / len(copies)  # bytes read (and written) per copy dispatch
    f_scale = known / (np.mean(copies) * 1024.0)
    w_scale = known / (np.mean(write["calibration_copy"]) * 1024.0)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    out = {}
    for k in sorted(set(fetch) & set(write)):
        if k.startswith(("sssp_", "spmv_", "tree_")):
            fb = float(np.mean(fetch[k])) * 1024.0 * f_scale
            wb = float(np.mean(write[k])) * 1024.0 * w_scale
            rec = {"kernel": k, "workload": workload, "dispatches": len(fetch[k]),
                   "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                   "hbm_bytes_per_launch": round(fb + wb), "fetch_scale": round(f_scale, 4),
                   "write_scale": round(w_scale, 4),
                   "calibration": f"{copy_mb} MiB elementwise copy (bitwise_not) x3, {len(copies)} dispatches "
                                  f"of {known / 2**20:.0f} MiB read + written each",
                   "command": command, "source_hash": source_hash()}
            with open(os.path.join(ROOT, "profiles", f"{k}_{workload}_pmc.json"), "w") as f:
                json.dump(rec, f, indent=1)
            out[k] = rec
    print(json.dumps(out, indent=1))


def run_pagerank(ctx, torch, synth, wc, stream, g, iters=10, reps=3):
    """PageRank sweeps over the in-edges of the scale-22 graph: per sweep 8 B
    per edge (source index, contribution gather) + 20 B per vertex (rank read,
    out-degree, contribution write, in-edge sum write and read, rank write)."""
    t = synth.transpose(g)
    dg = wc.DeviceCSR.from_host(t.row_ptr, t.col)
    od = torch.from_numpy(synth.out_degree(g)).cuda()
    del t
    r = torch.empty(g.n, dtype=torch.float32, device="cuda")
    alg = iters * (8.0 * g.m + 24.0 * g.n)
    res = {}
    for mode in ("flat", "wave", "block", "grid"):
        ctx.pagerank(dg, od, iters, mode=mode, out=r)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ctx.pagerank(dg, od, iters, mode=mode, out=r)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        res[mode] = {"ms": round(ms, 3), "sweep_ms": round(ms / iters, 4),
                     "gedges_s": round(iters * g.m / (ms * 1e-3) / 1e9, 2),
                     "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1)}
        print(f"[bench] pagerank {mode}: {res[mode]}", file=sys.stderr, flush=True)
    return {"workload": f"PageRank, damping 0.85, {iters} sweeps over the in-edges of the scale-22 R-MAT graph",
            "modes": res}


def run_coloring(ctx, torch, synth, wc, stream, g, reps=3):
    """Jones-Plassmann coloring (the GC benchmark) in every mode on a scale-16
    symmetric R-MAT graph shaped like the paper's Kron_log16 input, and on the
    symmetrized scale-22 graph (grid, wave and block: flat takes seconds there)."""
    out = {}
    for name, sg, modes in (("kron16", synth.symmetrize(synth.rmat_csr(16, 1 << 21)), ("flat", "wave", "block", "grid")),
                            ("rmat22", synth.symmetrize(g), ("wave", "block", "grid"))):
        dg = wc.DeviceCSR.from_host(sg.row_ptr, sg.col)
        dp = torch.from_numpy(synth.priorities(sg.n).view(np.int32)).cuda()
        col = torch.empty(sg.n, dtype=torch.int32, device="cuda")
        row = {"vertices": sg.n, "edges": sg.m}
        for mode in modes:
            _, st = ctx.color(dg, dp, mode=mode, out=col, stats=True)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                ctx.color(dg, dp, mode=mode, out=col)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            row[mode] = {"ms": round(ms, 3), "colors": st["rounds"], "us_per_round": round(1e3 * ms / st["rounds"], 1),
                         "gedges_s": round(2 * sg.m / (ms * 1e-3) / 1e9, 3)}
        out[name] = row
        print(f"[bench] coloring {name}: {row}", file=sys.stderr, flush=True)
        del dg, dp, col, sg
    return {"workload": "Jones-Plassmann coloring, seeded uint32 priorities, symmetric R-MAT graphs "
                        "(scale 16 with 2^21 sampled edges; the scale-22 graph symmetrized)",
            "note": "gedges_s counts each edge twice (count pass and release)", "results": out}


def run_ablation(ctx, torch, synth, wc, stream, scales=(12, 16), reps=3):
    """The paper's comparison against basic dynamic parallelism (Fig. 7, Fig. 8's
    launch counts), on this GPU: SSSP with one host-launched child per buffered
    vertex, SpMV with one per heavy row and tree descendants with one per
    internal node (tune driver 2, no consolidation) beside flat and the three
    consolidation levels, on smaller inputs (the per-item launches make the
    basic variant slow); and the allocator comparison (Fig. 5): SSSP's wave and
    block buffers in registers / LDS, in pool slices or from device malloc."""
    out = {}
    for scale in scales:
        g = synth.rmat_csr(scale, 16 << scale)
        w = synth.weights(g.m)
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        dw = torch.from_numpy(w.view(np.int32)).cuda()
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        row = {}
        for name, mode, tune in (("basic_dp", "grid", wc.make_tune(driver=2)), ("flat", "flat", None),
                                 ("wave", "wave", None), ("block", "block", None), ("grid", "grid", None),
                                 ("grid_1to1", "grid", wc.make_tune(driver=3))):
            _, st = ctx.sssp(dg, dw, 0, mode=mode, tune=tune, out=dist, stats=True)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                ctx.sssp(dg, dw, 0, mode=mode, tune=tune, out=dist)
            b.record(stream)
            torch.cuda.synchronize()
            row[name] = {"ms": round(a.elapsed_time(b) / reps, 3), "child_dispatches": st["dispatches"]}
        for name in ("flat", "wave", "block", "grid", "grid_1to1"):
            row[name]["speedup_vs_basic_dp"] = round(row["basic_dp"]["ms"] / row[name]["ms"], 1)
        out[f"rmat{scale}"] = row
        print(f"[bench] ablation scale {scale}: {row}", file=sys.stderr, flush=True)
        # allocator comparison (Sec. V.A, Fig. 5): the wave's / block's buffer in
        # registers / LDS, in a pool slice, or from device-side malloc per dispatch
        arow = {}
        for mode in ("wave", "block"):
            arow[mode] = {}
            for name, alloc in (("registers_lds", 0), ("pool", 1), ("device_malloc", 2)):
                tune = wc.make_tune(buffer_alloc=alloc)
                _, st = ctx.sssp(dg, dw, 0, mode=mode, tune=tune, out=dist, stats=True)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(reps):
                    ctx.sssp(dg, dw, 0, mode=mode, tune=tune, out=dist)
                b.record(stream)
                torch.cuda.synchronize()
                arow[mode][name] = {"ms": round(a.elapsed_time(b) / reps, 3), "fallback": bool(st["overflowed"])}
            arow[mode]["malloc_over_pool"] = round(arow[mode]["device_malloc"]["ms"] / arow[mode]["pool"]["ms"], 2)
            arow[mode]["basic_dp_over_pool"] = round(row["basic_dp"]["ms"] / arow[mode]["pool"]["ms"], 1)
        out[f"alloc_rmat{scale}"] = arow
        print(f"[bench] allocator comparison scale {scale}: {arow}", file=sys.stderr, flush=True)
        # SpMV on the same matrix: one child launch per heavy row (driver 2)
        val = torch.from_numpy(synth.values(g.m)).cuda()
        x = torch.from_numpy(synth.vector_x(g.n)).cuda()
        y = torch.empty(g.n, dtype=torch.float32, device="cuda")
        srow = {}
        for name, mode, tune in (("basic_dp", "grid", wc.make_tune(driver=2)), ("flat", "flat", None),
                                 ("wave", "wave", None), ("block", "block", None), ("grid", "grid", None)):
            _, st = ctx.spmv(dg, val, x, mode=mode, tune=tune, out=y, stats=True)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                ctx.spmv(dg, val, x, mode=mode, tune=tune, out=y)
            b.record(stream)
            torch.cuda.synchronize()
            srow[name] = {"ms": round(a.elapsed_time(b) / reps, 3), "child_dispatches": st["dispatches"]}
        for name in ("flat", "wave", "block", "grid"):
            srow[name]["speedup_vs_basic_dp"] = round(srow["basic_dp"]["ms"] / srow[name]["ms"], 1)
        out[f"spmv_rmat{scale}"] = srow
        print(f"[bench] ablation spmv scale {scale}: {srow}", file=sys.stderr, flush=True)
        # tree descendants on a random tree of the same size: one child launch per internal node
        t = synth.random_tree(1 << scale)
        dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
        desc = torch.empty(t.n, dtype=torch.int32, device="cuda")
        trow = {}
        for name, mode, tune in (("basic_dp", "grid", wc.make_tune(driver=2)), ("flat", "flat", None),
                                 ("wave", "wave", None), ("block", "block", None), ("grid", "grid", None)):
            _, st = ctx.tree_descendants(dt, mode=mode, tune=tune, out=desc, stats=True)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                ctx.tree_descendants(dt, mode=mode, tune=tune, out=desc)
            b.record(stream)
            torch.cuda.synchronize()
            trow[name] = {"ms": round(a.elapsed_time(b) / reps, 3), "child_dispatches": st["dispatches"]}
        for name in ("flat", "wave", "block", "grid"):
            trow[name]["speedup_vs_basic_dp"] = round(trow["basic_dp"]["ms"] / trow[name]["ms"], 1)
        out[f"td_tree{scale}"] = trow
        print(f"[bench] ablation tree descendants 2^{scale} nodes: {trow}", file=sys.stderr, flush=True)
    return {"workload": "SSSP from vertex 0 and SpMV on R-MAT graphs of 2^12 and 2^16 vertices, degree 16; "
                        "tree descendants on random trees of 2^12 and 2^16 nodes", "results": out}


def run_config_search(ctx, torch, synth, wc, stream, g, w, val, x, reps=3):
    """The configuration heuristic against exhaustive search (Sec. V.B compares
    KC_X with the best configuration found by search): grid mode of SSSP, SpMV and
    tree descendants on the headline inputs, every combination of workgroup size,
    items per lane, threshold and drain grid (resident maximum, or fewer
    workgroups as KC_X would give), against the library's defaults."""
    import itertools
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = torch.from_numpy(w.view(np.int32)).cuda()
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    dval, dx = torch.from_numpy(val).cuda(), torch.from_numpy(x).cuda()
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    t = synth.random_tree(1 << 22)
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    desc = torch.empty(t.n, dtype=torch.int32, device="cuda")
    calls = {"sssp": lambda tu: ctx.sssp(dg, dw, 0, mode="grid", tune=tu, out=dist),
             "spmv": lambda tu: ctx.spmv(dg, dval, dx, mode="grid", tune=tu, out=y),
             "tree_descendants": lambda tu: ctx.tree_descendants(dt, mode="grid", tune=tu, out=desc)}

    def timed(fn, tu):
        fn(tu)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn(tu)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {}
    for name, fn in calls.items():
        default_ms = timed(fn, None)
        best = (default_ms, "defaults")
        space = itertools.product((256, 512, 1024), (1, 2, 4, 8), (0, 4, 16, 32) if name != "tree_descendants"
                                  else (0,), (0, 512, 256, 128))
        tried = 0
        for block, ipl, th, gb in space:
            kw = dict(block_threads=block, items_per_lane=ipl)
            if th:
                kw["threshold"] = th
            if gb:
                kw["grid_blocks"] = gb
            ms = timed(fn, wc.make_tune(**kw))
            tried += 1
            if ms < best[0]:
                best = (ms, kw)
        out[name] = {"default_ms": round(default_ms, 4), "best_ms": round(best[0], 4), "best_config": best[1],
                     "default_vs_best": round(best[0] / default_ms, 3), "configs_tried": tried}
        print(f"[bench] config search {name}: {out[name]}", file=sys.stderr, flush=True)
    return {"workload": "grid mode on the scale-22 graph (SSSP from vertex 0, SpMV) and the 2^22-node tree "
                        "(descendants); grid_blocks 0 = resident maximum (KC_1)", "results": out}


def time_tree(ctx, torch, wc, stream, t, reps):
    """Every mode on one tree: descendants and heights, 20 B per node per pass
    (child_ptr, child, output, buffer entry), two passes (down and up) per call."""
    n = t.n
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {}
    for mode in ("flat", "wave", "block", "grid"):
        row = {}
        for what, fn in (("desc", ctx.tree_descendants), ("height", ctx.tree_height)):
            fn(dt, mode=mode, out=out)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn(dt, mode=mode, out=out)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            row[what + "_ms"] = round(ms, 4)
            row[what + "_gnodes_s"] = round(n / (ms * 1e-3) / 1e9, 3)
            row[what + "_alg_gbs"] = round(2 * 20.0 * n / (ms * 1e-3) / 1e9, 1)
        res[mode] = row
    return res


def run_trees(ctx, torch, synth, wc, stream, n=1 << 22, reps=5):
    """The 2^22-node random tree, and two fixed-depth trees in the manner of the
    paper's tree sets (Sec. V): fanout 128..256 with half of the inner nodes
    having children, and fanout 32..128 with all of them, each 4 levels deep."""
    out = {}
    for name, make, what in (
            ("random", lambda: synth.random_tree(n),
             f"random tree, {n} nodes, power-law fanout (alpha 2, max 4096), depth cap 24"),
            ("layered_half", lambda: synth.layered_tree(3, 128, 256, 0.5),
             "layered tree, 3 levels below the root, fanout 128..256, half of the inner nodes with children"),
            ("layered_full", lambda: synth.layered_tree(4, 32, 128, 1.0),
             "layered tree, 4 levels below the root, fanout 32..128, every inner node with children")):
        t = make()
        res = time_tree(ctx, torch, wc, stream, t, reps)
        out[name] = {"workload": what, "nodes": t.n, "modes": res}
        for mode, row in res.items():
            print(f"[bench] tree {name} {mode}: {row}", file=sys.stderr, flush=True)
        del t
    out["batch"] = run_tree_batch(ctx, torch, synth, wc, stream, reps)
    return out


def run_tree_batch(ctx, torch, synth, wc, stream, reps=5, count=64):
    """Batched trees: 64 random trees of 2^10..2^18 nodes in one call
    (wc_tree_descendants_batch / wc_tree_height_batch, grid and flat modes)
    against the same trees one call each."""
    trees = synth.batch_trees(count, 10.0, 18.0, seed=17)
    dts = [wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child) for t in trees]
    outs = [torch.empty(t.n, dtype=torch.int32, device="cuda") for t in trees]
    nodes = sum(t.n for t in trees)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {}
    for mode in ("flat", "grid"):
        for what, bfn, sfn in (("desc", ctx.tree_descendants_batch, ctx.tree_descendants),
                               ("height", ctx.tree_height_batch, ctx.tree_height)):
            one = timed(lambda: bfn(dts, mode=mode, outs=outs))
            each = timed(lambda: [sfn(d, mode=mode, out=o) for d, o in zip(dts, outs)])
            res[f"{mode}_{what}"] = {"batch_ms": round(one, 4), "one_call_per_tree_ms": round(each, 4),
                                     "speedup": round(each / one, 2),
                                     "batch_gnodes_s": round(nodes / (one * 1e-3) / 1e9, 3)}
            print(f"[bench] tree batch {mode} {what}: {res[f'{mode}_{what}']}", file=sys.stderr, flush=True)
    return {"workload": f"{count} random trees of 2^10..2^18 nodes ({nodes} nodes in total)", "modes": res}


def run_batch(args, ctx, torch, synth, wc):
    from paper_1606_08150_amd import autotune
    t0 = time.time()
    inst = synth.batch_instances(args.batch_count)
    graphs = [wc.DeviceCSR.from_host(g.row_ptr, g.col) for g, _ in inst]
    weights = [torch.from_numpy(w.view(np.int32)).cuda() for _, w in inst]
    degs = [torch.from_numpy(np.diff(g.row_ptr).astype(np.int64)).cuda() for g, _ in inst]
    srcs = [0] * len(inst)
    n_total = sum(g.n for g, _ in inst)
    m_total = sum(g.m for g, _ in inst)
    del inst
    print(f"[bench] batch of {len(graphs)} instances ({n_total} vertices, {m_total} edges) ready in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()

    def measure(modes, tunes, label):
        outs, st = ctx.sssp_batch(graphs, weights, srcs, modes=modes, tunes=tunes, stats=True)
        torch.cuda.synchronize()
        reached = sum(int(d[o != -1].sum().item()) for d, o in zip(degs, outs))
        rounds = st["rounds"] + 2
        ctx.sssp_batch(graphs, weights, srcs, modes=modes, tunes=tunes, outs=outs, graph_rounds=rounds)
        torch.cuda.synchronize()
        times = []
        for _ in range(args.batch_reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.sssp_batch(graphs, weights, srcs, modes=modes, tunes=tunes, outs=outs, graph_rounds=rounds)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        p50, p99 = float(np.percentile(times, 50)), float(np.percentile(times, 99))
        res = {"ms_p50": round(p50, 3), "ms_p99": round(p99, 3), "gteps": round(reached / (p50 * 1e-3) / 1e9, 3),
               "reached_edges": reached, "graph_rounds": rounds, "edges_relaxed": st["edges_processed"]}
        print(f"[bench] batch {label}: {res}", file=sys.stderr, flush=True)
        return res

    heur = measure(["grid"] * len(graphs), None, "heuristic")
    t1 = time.time()
    table = autotune.tune(ctx, graphs, weights, srcs, reps=2)
    tune_s = time.time() - t1
    modes, tunes = autotune.per_instance(table, [g.n for g in graphs])
    tuned = measure(modes, tunes, "tuned")
    return {"workload": f"{len(graphs)} R-MAT SSSP instances, 2^10..2^18 vertices log-uniform, degree 16, "
                        f"one graph-captured launch", "instances": len(graphs), "vertices": n_total,
            "edges": m_total, "heuristic": heur, "tuned": tuned, "table": table["buckets"],
            "block_threads": table["block_threads"], "autotune_s": round(tune_s, 1),
            "tuned_over_heuristic": round(heur["ms_p50"] / tuned["ms_p50"], 3)}


def run_serving(args, torch, synth, wc):
    from paper_1606_08150_amd import serve
    t0 = time.time()
    sizes = synth.serving_graph_sizes(64, 14, 20)
    dev, srcs, degs = [], [], []
    for k, n in enumerate(sizes):
        g, w, val, xs = synth.serving_graph(k, n, n_x=4)
        dev.append(serve.ResidentGraph(wc.DeviceCSR.from_host(g.row_ptr, g.col),
                                       torch.from_numpy(w.view(np.int32)).cuda(), torch.from_numpy(val).cuda(),
                                       [torch.from_numpy(x).cuda() for x in xs]))
        d = np.diff(g.row_ptr)
        srcs.append(np.flatnonzero(d > 0))
        degs.append(torch.from_numpy(d.astype(np.int64)).cuda())
    print(f"[bench] 64 resident graphs ({sum(sizes)} vertices) ready in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    ctx = wc.Context(0)
    reached_cache = {}

    def reached(gk, src):
        key = (gk, src)
        if key not in reached_cache:
            # through the batch entry point, so that the single-instance grid kernels'
            # per-launch profile stays that of the headline workload
            d = ctx.sssp_batch([dev[gk].csr], [dev[gk].w], [src], modes=["grid"])[0]
            reached_cache[key] = int(degs[gk][d != -1].sum().item())
        return reached_cache[key]

    rows = []
    backend = serve.GpuBackend(dev, sssp_mode=args.serve_sssp_mode)
    srv = serve.Server(backend, workers=args.serve_workers, max_slots=512, max_batch=64)
    try:
        warm = serve.poisson_requests(200, 5000.0, srcs, n_x=4, seed=1)
        srv.run(warm)
        for rate in [float(x) for x in args.serve_rates.split(",")]:
            reqs = serve.poisson_requests(args.serve_requests, rate, srcs, n_x=4, seed=int(rate))
            out = srv.run(reqs, time_limit=300)
            edges = sum(reached(r.graph, r.arg) for r in out if r.kind == serve.SSSP)
            row = {"rate_rps": rate, **serve.summarize(out, edges), "pool_growths": srv.grows,
                   "pool_growth_bytes": srv.admission.pool_growth, "peak_used_bytes": srv.admission.peak_used,
                   "budget_bytes": srv.admission.budget}
            rows.append(row)
            print(f"[bench] serving {row}", file=sys.stderr, flush=True)
    finally:
        srv.close()
        ctx.close()
    return {"workload": "Poisson arrivals, 50% SSSP (random source with out-edges) / 50% SpMV (4 resident x "
                        "per graph), 64 resident R-MAT graphs of 2^14..2^20 vertices, degree 16",
            "workers": args.serve_workers, "sssp_mode": args.serve_sssp_mode, "graphs_vertices": sum(sizes),
            "requests_per_rate": args.serve_requests,
            "admission": "outputs by exact tensor bytes; batch workspace from the library's plan-only mode "
                         "against each worker's pool; pool growth charged to the budget (half the free memory "
                         "measured after the workers' contexts exist)",
            "rates": rows}


def main():
    if "--summarize-kernel-stats" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-kernel-stats", action="store_true")
        sp.add_argument("--stats-csv", required=True)
        sp.add_argument("--workload", required=True)
        sp.add_argument("--command", required=True)
        sp.add_argument("--out-name", required=True)
        a = sp.parse_args()
        summarize_kernel_stats(a.stats_csv, a.workload, a.command, a.out_name)
        return
    if "--summarize-counters" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-counters", action="store_true")
        sp.add_argument("--sq-dir", required=True)
        sp.add_argument("--tcc-dir", required=True)
        sp.add_argument("--workload", default="rmat22")
        sp.add_argument("--command", required=True)
        sp.add_argument("--out-name", required=True)
        sp.add_argument("--cyc-dir", default=None)
        sp.add_argument("--cyc-command", default=None)
        a = sp.parse_args()
        summarize_counters(a.sq_dir, a.tcc_dir, a.workload, a.command, a.out_name, cyc_dir=a.cyc_dir,
                           cyc_command=a.cyc_command)
        return
    if "--summarize-mode-counters" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-mode-counters", action="store_true")
        sp.add_argument("--run", action="append", required=True, help="MODE=DIR (repeatable)")
        sp.add_argument("--workload", default="rmat22")
        sp.add_argument("--command", required=True)
        sp.add_argument("--out-name", required=True)
        a = sp.parse_args()
        runs = {}
        for item in a.run:
            mode, d = item.split("=", 1)
            runs.setdefault(mode, []).append(d)
        summarize_mode_counters(runs, a.workload, a.command, a.out_name)
        return
    if "--summarize-profiles" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-profiles", action="store_true")
        sp.add_argument("--fetch-dir", required=True)
        sp.add_argument("--write-dir", required=True)
        sp.add_argument("--copy-mb", type=int, required=True)
        sp.add_argument("--workload", default="rmat22")
        sp.add_argument("--command", required=True)
        sp.add_argument("--stats-csv", default=None)
        sp.add_argument("--stats-command", default=None)
        sp.add_argument("--stats-name", default=None)
        a = sp.parse_args()
        summarize_profiles(a.fetch_dir, a.write_dir, a.copy_mb, a.workload, a.command)
        if a.stats_csv:
            summarize_kernel_stats(a.stats_csv, a.workload, a.stats_command, a.stats_name)
        return
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

    if args.calibrate_copy_mb > 0:
        # a plain elementwise copy with a unique kernel name (bitwise_not: one
        # 4-byte read and one 4-byte write per element)
        nb = args.calibrate_copy_mb << 20
        src_buf = torch.zeros(nb // 4, dtype=torch.int32, device="cuda")
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.bitwise_not(src_buf, out=dst_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
        print(f"[bench] calibration copy: 3 x {args.calibrate_copy_mb} MiB", file=sys.stderr, flush=True)

    ctx = wc.Context(0)
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = torch.from_numpy(w.view(np.int32)).cuda()
    dval, dx = torch.from_numpy(val).cuda(), torch.from_numpy(x).cuda()
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    if args.counter_run:
        # counter passes per mode: SSSP, SpMV and tree descendants, 3 calls each
        t = synth.random_tree(1 << 22)
        dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
        out_t = torch.empty(t.n, dtype=torch.int32, device="cuda")
        y = torch.empty(g.n, dtype=torch.float32, device="cuda")
        mode = args.counter_run
        times = {}
        for name, fn in (("sssp", lambda: ctx.sssp(dg, dw, 0, mode=mode, out=dist)),
                         ("spmv", lambda: ctx.spmv(dg, dval, dx, mode=mode, out=y)),
                         ("tree", lambda: ctx.tree_descendants(dt, mode=mode, out=out_t))):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            times[name] = round((time.perf_counter() - t1) / 3 * 1e3, 3)
        print(json.dumps({"counter_run": mode, "ms_per_call": times}), flush=True)
        ctx.close()
        return
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    deg = torch.from_numpy(np.diff(g.row_ptr).astype(np.int64)).cuda()
    stream = torch.cuda.current_stream()

    def sssp(mode):
        ctx.sssp(dg, dw, 0, mode=mode, out=dist)

    def spmv(mode):
        ctx.spmv(dg, dval, dx, mode=mode, out=y)

    def bfs(mode):
        ctx.bfs(dg, 0, mode=mode, out=dist)

    # reached edges (GTEPS numerator) from the GPU result: out-edges of vertices with finite distance
    sssp(args.mode)
    torch.cuda.synchronize()
    reached_mask = dist != -1  # INF as int32
    m_reached = int(deg[reached_mask].sum().item())
    n_reached = int(reached_mask.sum().item())
    # per-call work counters (outside the timed region)
    _, sst = ctx.sssp(dg, dw, 0, mode=args.mode, out=dist, stats=True)

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
    sssp_thr = wc.default_tune("sssp", args.mode, 1)["threshold"]
    reached_np = reached_mask.cpu().numpy()
    sheavy = reached_np & (lens > sssp_thr)
    slight = reached_np & ~(lens > sssp_thr)
    info = dict(n=g.n, nnz_heavy=int(lens[heavy].sum()), rows_heavy=int(heavy.sum()),
                nnz_light=int(lens[~heavy].sum()), sssp_edges=sst["edges_processed"],
                sssp_edges_buffered=sst["edges_buffered"], sssp_updates=sst["updates"],
                sssp_updates_buffered=sst["updates_buffered"], sssp_rounds=sst["rounds"], sssp_calls=args.steps,
                reached_edges_heavy=int(lens[sheavy].sum()), reached_heavy=int(sheavy.sum()),
                reached_edges_light=int(lens[slight].sum()), reached_light=int(slight.sum()))
    workload_tag = f"rmat{scale}"
    dominant = max(ktimes.items(), key=lambda kv: kv[1][1])
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 4), "avg_ms": round(v[1] / v[0], 5)}
               for k, v in sorted(ktimes.items(), key=lambda kv: -kv[1][1])}
    def roof(name):
        launches, total, _ = ktimes[name]
        ab = algorithmic_bytes(name, info, launches)
        if ab is None:
            return None
        bytes_per_launch, what = ab
        avg_s = total / launches * 1e-3
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = counter_traffic(name, workload_tag)
        return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic is not None else None,
                "bytes_per_launch": round(bytes_per_launch), "bytes_model": what,
                "launches": launches, "avg_launch_ms": round(total / launches, 5)}

    roofline = roof(dominant[0])
    spmv_roofline = roof("spmv_drain") if "spmv_drain" in ktimes else None

    # ---- attainable HBM bandwidth on this GPU: a plain 1 GiB device copy (read +
    # write bytes over the event-timed copy), reported beside the published peak
    src_c = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    dst_c = torch.empty_like(src_c)
    dst_c.copy_(src_c)
    torch.cuda.synchronize()
    a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a_ev.record(stream)
    for _ in range(5):
        dst_c.copy_(src_c)
    b_ev.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src_c.numel() * 4 * 5 / (a_ev.elapsed_time(b_ev) * 1e-3) / 1e9
    del src_c, dst_c
    for rl in (roofline, spmv_roofline):
        if rl is not None:
            rl["attainable_copy"] = round(copy_gbs, 1)
            rl["frac_of_attainable"] = round(rl["achieved"] / copy_gbs, 4)

    # ---- cold caches: each call after a 512 MiB write that evicts L2 and MALL
    cold = None
    if not args.no_cold:
        flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        cold = {}
        for prob, fn in (("sssp", sssp), ("spmv", spmv)):
            times = []
            for _ in range(5):
                flush.fill_(1)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn(args.mode)
                b.record(stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b))
            cold[prob + "_ms_median"] = round(float(np.median(times)), 4)
        del flush
        print(f"[bench] cold caches: {cold}", file=sys.stderr, flush=True)

    # ---- context for the drains: a bare gather of x over the same CSR columns
    # (torch.index_select, int64 indices), and over the columns sorted (the same
    # bytes with perfect locality); untimed for `value`
    gather_ceiling = None
    if not args.no_gather_ceiling:
        col64 = torch.from_numpy(g.col.astype(np.int64)).cuda()
        gout = torch.empty(g.m, dtype=torch.float32, device="cuda")

        def timed_gather(idx, reps=10):
            torch.index_select(dx, 0, idx, out=gout)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                torch.index_select(dx, 0, idx, out=gout)
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        gather_ceiling = {"what": f"torch.index_select of x over the {g.m} CSR columns",
                          "csr_order_ms": round(timed_gather(col64), 4)}
        col64 = torch.sort(col64).values
        gather_ceiling["sorted_ms"] = round(timed_gather(col64), 4)
        del col64, gout
        print(f"[bench] gather ceiling: {gather_ceiling}", file=sys.stderr, flush=True)

    # ---- the hot-column layout (wc_spmv_prepare once, then wc_spmv_hot per
    # product, its gather of the hot x values included): grid mode, bit-identical
    # to wc_spmv; untimed for `value`
    spmv_hot = None
    if not args.no_spmv_hot:
        y_hot = torch.empty(g.n, dtype=torch.float32, device="cuda")
        spmv_hot = {"what": "wc_spmv_hot in grid mode after wc_spmv_prepare (columns ranked by use; the hot "
                            "x values gathered per product, the most used staged in LDS by the drain)",
                    "by_hot": {}}
        for hot in (16384, 65536, 262144):
            t1 = time.perf_counter()
            a_hot, ids = ctx.spmv_prepare(dg, hot)
            prep_s = time.perf_counter() - t1
            ctx.spmv_hot(a_hot, ids, dval, dx, mode="grid", out=y_hot)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(10):
                ctx.spmv_hot(a_hot, ids, dval, dx, mode="grid", out=y_hot)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / 10
            spmv_hot["by_hot"][str(hot)] = {"ms": round(ms, 4), "alg_gbs": round(spmv_bytes / (ms * 1e-3) / 1e9, 1),
                                            "frac_hbm": round(spmv_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                            "prepare_s": round(prep_s, 3)}
            del a_hot, ids
        best = min(spmv_hot["by_hot"].items(), key=lambda kv: kv[1]["ms"])
        spmv_hot["best_hot"] = int(best[0])
        spmv_hot["speedup_vs_wc_spmv"] = round(spmv_avg / best[1]["ms"], 3)
        print(f"[bench] spmv hot-column layout: {spmv_hot}", file=sys.stderr, flush=True)

    # ---- flat / wave / block / grid side by side (mean of 3 calls after 1 warm-up)
    modes = {}
    if not args.no_modes:
        for mode in ("flat", "wave", "block", "grid"):
            res = {}
            for prob, fn in (("sssp", sssp), ("spmv", spmv), ("bfs", bfs)):
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
            # BFS from vertex 0 reaches the same vertices as the SSSP: same edge count
            res["bfs_gteps"] = round(m_reached / (res["bfs_ms"] * 1e-3) / 1e9, 3)
            modes[mode] = res
            print(f"[bench] mode {mode}: {res}", file=sys.stderr, flush=True)

    # ---- PageRank on the same graph (in-edges), 10 sweeps, every mode
    pagerank = None
    if not args.no_pagerank:
        pagerank = run_pagerank(ctx, torch, synth, wc, stream, g)

    # ---- graph coloring (Jones-Plassmann), every mode
    coloring = None
    if not args.no_coloring:
        coloring = run_coloring(ctx, torch, synth, wc, stream, g)

    # ---- consolidated vs basic dynamic parallelism (per-vertex child launches)
    ablation = None
    if not args.no_ablation:
        ablation = run_ablation(ctx, torch, synth, wc, stream)

    # ---- the configuration heuristic against exhaustive search (grid mode)
    config_search = None
    if not args.no_config_search:
        config_search = run_config_search(ctx, torch, synth, wc, stream, g, w, val, x)

    # ---- trees: descendants and heights on the 2^22-node random tree, every mode
    trees = None
    if not args.no_trees:
        trees = run_trees(ctx, torch, synth, wc, stream)

    # ---- batched SSSP: 512 independent R-MAT instances (2^10..2^18 vertices,
    # degree 16) in one graph-captured launch; heuristic vs autotuned per bucket
    batch = None
    if not args.no_batch:
        batch = run_batch(args, ctx, torch, synth, wc)

    # ---- serving: Poisson streams of SSSP/SpMV requests over 64 resident graphs
    serving = None
    if not args.no_serve:
        serving = run_serving(args, torch, synth, wc)

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
        # context: the oracle's fp64 SpMV on the same matrix, one core and all
        # host threads (row blocks side by side), and the host
        t1 = time.perf_counter()
        oracle.spmv_f64(g.row_ptr, g.col, val, x)
        cpu["spmv_f64_s"] = round(time.perf_counter() - t1, 3)
        threads = min(os.cpu_count() or 1, 16)
        oracle.spmv_f64_threads(g.row_ptr, g.col, val, x, threads)
        t1 = time.perf_counter()
        for _ in range(3):
            oracle.spmv_f64_threads(g.row_ptr, g.col, val, x, threads)
        cpu["spmv_f64_all_threads_s"] = round((time.perf_counter() - t1) / 3, 4)
        cpu["spmv_f64_threads"] = threads
        # the batch (C4 protocol: instances side by side, one per host thread):
        # the first 128 instances of the 512-instance batch (counter-based
        # generator: the same instances), one Dijkstra each
        import concurrent.futures as cf
        inst = synth.batch_instances(128)

        def one(gw):
            d_ = oracle.sssp_dijkstra(gw[0].row_ptr, gw[0].col, gw[1], 0)
            return oracle.sssp_reached_edges(gw[0].row_ptr, d_)
        t1 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            reached_b = sum(ex.map(one, inst))
        dtb = time.perf_counter() - t1
        cpu["batch_sample"] = {"instances": len(inst), "vertices": sum(gw[0].n for gw in inst),
                               "edges": sum(gw[0].m for gw in inst), "s": round(dtb, 3),
                               "gteps": round(reached_b / dtb / 1e9, 4), "threads": threads}
        del inst
        # trees: descendants and heights of the 2^22-node random tree, one core
        tr = synth.random_tree(1 << 22)
        t1 = time.perf_counter()
        oracle.tree_descendants(tr.child_ptr, tr.child)
        cpu["tree_desc_s"] = round(time.perf_counter() - t1, 3)
        t1 = time.perf_counter()
        oracle.tree_height(tr.child_ptr, tr.child)
        cpu["tree_height_s"] = round(time.perf_counter() - t1, 3)
        del tr
        cpu["host_cpu"] = host_cpu_model()
        cpu["host_threads"] = os.cpu_count()

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
        "spmv_roofline": spmv_roofline,
        "gather_ceiling": gather_ceiling,
        "spmv_hot": spmv_hot,
        "cold_caches": cold,
        "sssp_work": {"edges_relaxed": sst["edges_processed"], "edges_by_consolidated_child": sst["edges_buffered"],
                      "relaxations_per_reachable_edge": round(sst["edges_processed"] / max(m_reached, 1), 4),
                      "updates": sst["updates"], "updates_by_consolidated_child": sst["updates_buffered"],
                      "rounds": sst["rounds"], "items_buffered": sst["items_buffered"]},
        "kernels": kernels,
        "modes": modes,
        "pagerank": pagerank,
        "coloring": coloring,
        "basic_dp_ablation": ablation,
        "config_search": config_search,
        "trees": trees,
        "batch": batch,
        "serving": serving,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    ctx.close()
    line = json.dumps(out)
    print(line, flush=True)
    if args.jsonl:
        with open(args.jsonl, "a") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
