"""The C-ABI library loads on the CPU and exports every symbol include/wc.h declares;
its host-side planning helpers agree with the oracle and the cited fixtures."""
import os
import re

import oracle

from paper_1606_08150_amd import wc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "wc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = wc.load_library()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(wc.EXPORTS)


def test_version_string():
    assert b"gfx950" in wc.load_library().wc_version()


def test_host_helpers_match_oracle():
    for args in [(256, 1, 4), (64, 3, 4), (1, 1, 1), (1024, 2, 8)]:
        assert wc.per_buffer_size(*args) == oracle.per_buffer_size(*args)
    for args in [(26, 1024, 1), (26, 1024, 16), (208, 256, 32), (1, 64, 32), (2048, 256, 16)]:
        assert wc.kc_config(*args) == oracle.kc_config(*args)


def test_default_tune_and_errors():
    t = wc.default_tune("sssp", "grid", 2048)
    assert t["grid_blocks"] == 2048 and t["items_per_lane"] == 2 and t["block_threads"] == 512
    # SSSP and SpMV wave and block levels: short items inline, chunks of 128
    for problem in ("sssp", "spmv"):
        for mode in ("wave", "block"):
            t = wc.default_tune(problem, mode, 2048)
            assert (t["threshold"], t["items_per_lane"], t["block_threads"]) == (8, 2, 256)
    assert wc.default_tune("bfs", "wave", 1)["threshold"] == 32
    # the packet queues: larger workgroups
    assert wc.default_tune("bfs", "wave", 1)["block_threads"] == 1024
    assert wc.default_tune("bfs", "block", 1)["block_threads"] == 512
    assert wc.default_tune("tree", "wave", 1)["block_threads"] == 1024
    assert wc.default_tune("tree", "block", 1)["block_threads"] == 256
    assert wc.default_tune("spmv", "grid", 1)["items_per_lane"] == 8
    # BFS: grid rounds share SSSP's chunk, the recursion queue packs coarser
    assert wc.default_tune("bfs", "grid", 1)["items_per_lane"] == 2
    assert wc.default_tune("bfs", "wave", 1)["items_per_lane"] == 64
    assert wc.default_tune("bfs", "block", 1)["items_per_lane"] == 32
    assert wc.default_tune("tree", "wave", 1)["items_per_lane"] == 32
    assert wc.default_tune("tree", "grid", 1)["items_per_lane"] == 2
    assert wc.default_tune("tree", "block", 100)["threshold"] == 0
    t = wc.default_tune("tree", "grid", 100)
    assert t["block_threads"] == 512 and t["items_per_lane"] == 2
    t = wc.default_tune("color", "grid", 100)
    assert t["threshold"] == 64 and t["block_threads"] == 256 and t["items_per_lane"] == 2
    assert wc.default_tune("color", "wave", 100)["threshold"] == 32
    # coloring in wave and block modes: chunks of 64, the block child from 8
    for mode, thr in (("wave", 32), ("block", 8)):
        t = wc.default_tune("color", mode, 100)
        assert (t["threshold"], t["items_per_lane"]) == (thr, 1)
    try:
        wc.default_tune("nope", "grid", 1)
    except wc.WcError as e:
        assert e.status == -1
    else:
        raise AssertionError("unknown problem accepted")


def test_spmv_noalloc_refuses_before_touching_the_device():
    """The no-allocation SpMV checks its size limit and tune on the host, before
    any HIP call (so this runs without a GPU; no pointer is dereferenced)."""
    import ctypes
    lib = wc.load_library()
    dummy = 256  # never dereferenced: every call below is refused first
    big = wc.CCsr(1 << 22, 1 << 26, dummy, dummy)
    assert lib.wc_spmv_noalloc(ctypes.byref(big), dummy, dummy, dummy, wc.GRID, None, None) == -1
    assert b"exceeds the fixed scratch" in lib.wc_last_error()
    small = wc.CCsr(1000, 4000, dummy, dummy)
    t = wc.make_tune(driver=2)
    assert lib.wc_spmv_noalloc(ctypes.byref(small), dummy, dummy, dummy, wc.GRID, ctypes.byref(t), None) == -1
    assert lib.wc_spmv_noalloc(ctypes.byref(small), dummy, dummy, dummy, 7, None, None) == -1
    assert lib.wc_spmv_noalloc(ctypes.byref(small), None, dummy, dummy, wc.GRID, None, None) == -1
    empty = wc.CCsr(0, 0, None, None)
    assert lib.wc_spmv_noalloc(ctypes.byref(empty), None, None, None, wc.GRID, None, None) == 0
