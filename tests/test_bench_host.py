"""Host logic of bench.py (CPU only): the one-GPU guard, the algorithmic-byte
models behind the roofline, the counter-file lookup keyed by the kernel sources,
and the kernel-trace summary."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_models():
    info = {"sssp_edges_buffered": 1000, "sssp_updates_buffered": 10, "sssp_calls": 3, "sssp_edges": 1200,
            "sssp_updates": 15, "n": 50, "sssp_rounds": 4, "nnz_heavy": 700, "rows_heavy": 7, "nnz_light": 300,
            "reached_edges_heavy": 900, "reached_heavy": 20, "reached_edges_light": 150, "reached_light": 30}
    b, _ = bench.algorithmic_bytes("sssp_drain", info, 6)
    assert b == (16 * 900 + 20 * 20) * 3 / 6  # each reachable edge once, however often it is relaxed
    b, _ = bench.algorithmic_bytes("sssp_round_grid", info, 12)
    assert b == (16 * 150 + 20 * 30) * 3 / 12
    more = dict(info, sssp_edges_buffered=5000)  # redundant relaxations add no useful bytes
    assert bench.algorithmic_bytes("sssp_drain", more, 6)[0] == (16 * 900 + 20 * 20) * 3 / 6
    assert bench.algorithmic_bytes("spmv_drain", info, 1)[0] == 12 * 700 + 4 * 7
    assert bench.algorithmic_bytes("spmv_parent_grid", info, 1)[0] == 12 * 300 + 8 * 50
    assert bench.algorithmic_bytes("something_else", info, 1) is None


def test_counter_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1606_08150_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.source_hash()
    rec = {"kernel": "sssp_drain", "hbm_bytes_per_launch": 1234, "source_hash": h}
    (tmp_path / "profiles" / "sssp_drain_w_pmc.json").write_text(json.dumps(rec))
    assert bench.counter_traffic("sssp_drain", "w") == 1234
    assert bench.counter_traffic("spmv_drain", "w") is None  # no file
    (csrc / "k.hip").write_text("// kernel v2\n")  # sources changed since the counters were taken
    assert bench.source_hash() != h
    assert bench.counter_traffic("sssp_drain", "w") is None


def test_kernel_stats_summary(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    csv_path = tmp_path / "stats.csv"
    csv_path.write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs,StdDev\n"
        "\"void wc::(anonymous namespace)::sssp_drain<512>(wc::(anonymous namespace)::SsspArgs, int)\","
        "10,1000000,100000,75.0,3000,600000,1\n"
        "\"wc::zero_stats(wc::DevStats*)\",5,10000,2000,25.0,1900,2100,1\n")
    bench.summarize_kernel_stats(str(csv_path), "w", "rocprofv3 --kernel-trace --stats -- python3 bench.py", "ks_w")
    text = (tmp_path / "profiles" / "ks_w.md").read_text()
    assert "rocprofv3 --kernel-trace --stats -- python3 bench.py" in text
    row = next(line for line in text.splitlines() if line.startswith("| sssp_drain"))
    cells = [c.strip() for c in row.split("|")]
    assert cells[2] == "10" and cells[3] == "100.00" and cells[6] == "1.000"
    assert any(line.startswith("| zero_stats") for line in text.splitlines())


@pytest.mark.parametrize("name,short", [
    ("void wc::(anonymous namespace)::color_round_grid<256>(wc::(anonymous namespace)::ColorArgs, int)",
     "color_round_grid"),
    ("wc::zero_stats(wc::DevStats*)", "zero_stats"),
])
def test_short_kernel_names(name, short):
    assert bench._short_kernel(name) == short


def test_counter_summary(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    head = ("Correlation_Id,Dispatch_Id,Agent_Id,Queue_Id,Process_Id,Thread_Id,Grid_Size,Kernel_Id,Kernel_Name,"
            "Workgroup_Size,LDS_Block_Size,Scratch_Size,VGPR_Count,Accum_VGPR_Count,SGPR_Count,Counter_Name,"
            "Counter_Value,Start_Timestamp,End_Timestamp\n")
    name = "\"void wc::(anonymous namespace)::sssp_drain<512>(wc::(anonymous namespace)::SsspArgs, int)\""

    def row(disp, counter, value):
        return f"1,{disp},A,1,1,1,512,1,{name},512,0,0,24,0,16,{counter},{value},0,1\n"
    sq, tcc = tmp_path / "sq", tmp_path / "tcc"
    sq.mkdir()
    tcc.mkdir()
    (sq / "run_counter_collection.csv").write_text(
        head + row(1, "SQ_WAVES", 100) + row(1, "SQ_INSTS_VALU", 5000) + row(1, "SQ_WAVE_CYCLES", 4000)
        + row(2, "SQ_WAVES", 100) + row(2, "SQ_INSTS_VALU", 3000) + row(2, "SQ_WAVE_CYCLES", 4000))
    (tcc / "run_counter_collection.csv").write_text(
        head + row(1, "TCC_HIT_sum", 30) + row(1, "TCC_MISS_sum", 10) + row(1, "TCC_ATOMIC_sum", 8)
        + row(2, "TCC_HIT_sum", 30) + row(2, "TCC_MISS_sum", 30) + row(2, "TCC_ATOMIC_sum", 4))
    bench.summarize_counters(str(sq), str(tcc), "w", "cmd", "ctr_w", with_static=False)
    line = next(x for x in (tmp_path / "profiles" / "ctr_w.md").read_text().splitlines()
                if x.startswith("| sssp_drain"))
    cells = [c.strip() for c in line.split("|")][1:-1]
    # dispatches, waves, VALU per wave, wave-cycles per wave, L2 hit rate, atomics per dispatch
    assert cells[1] == "2" and cells[3] == "200" and cells[4] == "40.00" and cells[6] == "40.00"
    assert cells[9] == "0.60" and cells[10] == "6"


def test_mode_counter_summary(tmp_path, monkeypatch):
    """Per-mode counters (the Figs. 8-10 analogue): lane utilization from the
    summed VALU thread cycles, occupancy weighted by dispatch cycles, bytes per
    call from the calibrated FETCH_SIZE plus WRITE_SIZE; kernels are grouped by
    problem from their names."""
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    head = ("Correlation_Id,Dispatch_Id,Agent_Id,Queue_Id,Process_Id,Thread_Id,Grid_Size,Kernel_Id,Kernel_Name,"
            "Workgroup_Size,LDS_Block_Size,Scratch_Size,VGPR_Count,Accum_VGPR_Count,SGPR_Count,Counter_Name,"
            "Counter_Value,Start_Timestamp,End_Timestamp\n")

    def row(disp, kernel, counter, value):
        name = f"\"void wc::(anonymous namespace)::{kernel}<256>(wc::(anonymous namespace)::Args)\""
        return f"1,{disp},A,1,1,1,512,1,{name},256,0,0,24,0,16,{counter},{value},0,1\n"
    sq, fe, wr = tmp_path / "sq", tmp_path / "fe", tmp_path / "wr"
    for d in (sq, fe, wr):
        d.mkdir()
    (sq / "run_counter_collection.csv").write_text(
        head + row(1, "sssp_round", "SQ_THREAD_CYCLES_VALU", 3200) + row(1, "sssp_round", "SQ_ACTIVE_INST_VALU", 100)
        + row(1, "sssp_round", "SQ_INSTS_VALU", 300) + row(1, "sssp_round", "GRBM_GUI_ACTIVE", 1000)
        + row(1, "sssp_round", "MeanOccupancyPerCU", 10)
        + row(2, "sssp_drain", "SQ_THREAD_CYCLES_VALU", 6400) + row(2, "sssp_drain", "SQ_ACTIVE_INST_VALU", 100)
        + row(2, "sssp_drain", "GRBM_GUI_ACTIVE", 3000) + row(2, "sssp_drain", "MeanOccupancyPerCU", 20)
        + row(3, "zero_stats", "SQ_INSTS_VALU", 99))
    (fe / "run_counter_collection.csv").write_text(head + row(1, "sssp_round", "FETCH_SIZE", 1000))
    (wr / "run_counter_collection.csv").write_text(head + row(1, "sssp_drain", "WRITE_SIZE", 1000))
    bench.summarize_mode_counters({"wave": [str(sq), str(fe), str(wr)]}, "w", "cmd", "modes_w")
    line = next(x for x in (tmp_path / "profiles" / "modes_w.md").read_text().splitlines()
                if x.startswith("| sssp | wave"))
    cells = [c.strip() for c in line.split("|")][1:-1]
    # VALU per call 300 / 3; utilization (3200 + 6400) / (64 x 200) = 0.75;
    # occupancy (10 x 1000 + 20 x 3000) / 4000 = 17.5; bytes (2 x 1000 + 1000) KiB / 3
    assert cells[2] == "100" and cells[3] == "0.750" and cells[4] == "17.5"
    assert cells[5] == f"{3000 * 1024 / 3 / 1e6:.1f}"
