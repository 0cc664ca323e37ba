"""Oracle: plain CPU implementations of what the consolidation hot path computes.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1606_08150_amd``) and neither imports the
other; the only common dependency is the seeded input module ``synth``.

The arithmetic lives in ``oracle.c`` (see its header for what each function
follows in the paper); this module marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
INF = np.uint32(0xFFFFFFFF)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing; run oracle.build.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    c = ctypes
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    pi64 = c.POINTER(c.c_int64)
    sig = {
        "orc_sssp_dijkstra": (c.c_int, [c.c_int32, i32p, i32p, u32p, c.c_int32, u32p]),
        "orc_sssp_bellman_ford": (c.c_int, [c.c_int32, i32p, i32p, u32p, c.c_int32, u32p]),
        "orc_sssp_certify": (c.c_int, [c.c_int32, i32p, i32p, u32p, c.c_int32, u32p, pi64]),
        "orc_sssp_reached_edges": (c.c_int64, [c.c_int32, i32p, u32p]),
        "orc_spmv_f64": (None, [c.c_int32, i32p, i32p, f32p, f32p, f64p, f64p]),
        "orc_spmv_check": (c.c_int64, [c.c_int32, f64p, f64p, f32p, c.c_double, pi64]),
        "orc_pagerank_f64": (c.c_int, [c.c_int32, i32p, i32p, i32p, c.c_int32, c.c_double, f64p]),
        "orc_bfs": (c.c_int, [c.c_int32, i32p, i32p, c.c_int32, u32p]),
        "orc_color_jp": (c.c_int32, [c.c_int32, i32p, i32p, u32p, i32p]),
        "orc_color_certify": (c.c_int64, [c.c_int32, i32p, i32p, u32p, i32p, pi64]),
        "orc_tree_validate": (c.c_int, [c.c_int32, i32p, i32p, i32p]),
        "orc_tree_descendants": (c.c_int, [c.c_int32, i32p, i32p, i32p]),
        "orc_tree_height": (c.c_int, [c.c_int32, i32p, i32p, i32p]),
        "orc_tree_descendants_brute": (c.c_int, [c.c_int32, i32p, i32p]),
        "orc_tree_height_brute": (c.c_int, [c.c_int32, i32p, i32p]),
        "orc_count_heavy": (c.c_int64, [c.c_int64, i64p, c.c_int64]),
        "orc_consolidation_plan": (None, [c.c_int64, i64p, c.c_int64, c.c_int64, pi64, pi64, pi64, pi64]),
        "orc_per_buffer_size": (c.c_int64, [c.c_int64, c.c_int64, c.c_int64]),
        "orc_kc_config": (None, [c.c_int64, c.c_int64, c.c_int64, pi64, pi64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _nonempty(a, dtype):
    """ctypes ndpointer rejects nothing for empty arrays, but give C a valid address."""
    a = np.ascontiguousarray(a, dtype=dtype)
    return a if a.size else np.zeros(1, dtype=dtype)


# ---- SSSP ---------------------------------------------------------------------------------------

def sssp_dijkstra(row_ptr, col, w, src: int) -> np.ndarray:
    n = len(row_ptr) - 1
    dist = np.empty(max(n, 1), dtype=np.uint32)
    rc = _load().orc_sssp_dijkstra(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(w, np.uint32), src, dist)
    if rc != 0:
        raise ValueError(f"orc_sssp_dijkstra failed ({rc})")
    return dist[:n]


def sssp_bellman_ford(row_ptr, col, w, src: int) -> np.ndarray:
    n = len(row_ptr) - 1
    dist = np.empty(max(n, 1), dtype=np.uint32)
    rc = _load().orc_sssp_bellman_ford(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(w, np.uint32), src,
                                       dist)
    if rc != 0:
        raise ValueError(f"orc_sssp_bellman_ford failed ({rc})")
    return dist[:n]


def sssp_certify(row_ptr, col, w, src: int, dist):
    """(code, where): code 0 = dist is the exact shortest-path vector; see oracle.c."""
    n = len(row_ptr) - 1
    where = ctypes.c_int64(-1)
    rc = _load().orc_sssp_certify(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(w, np.uint32), src,
                                  _nonempty(dist, np.uint32), ctypes.byref(where))
    return rc, where.value


def sssp_reached_edges(row_ptr, dist) -> int:
    n = len(row_ptr) - 1
    return int(_load().orc_sssp_reached_edges(n, _i32(row_ptr), _nonempty(dist, np.uint32)))


# ---- SpMV ---------------------------------------------------------------------------------------

def bfs(row_ptr, col, src: int):
    """Breadth-first levels (uint32, INF unreachable)."""
    n = len(row_ptr) - 1
    lv = np.empty(max(n, 1), dtype=np.uint32)
    if _load().orc_bfs(n, _i32(row_ptr), _nonempty(col, np.int32), int(src), lv) != 0:
        raise MemoryError("orc_bfs")
    return lv[:n]


def color_jp(row_ptr, col, prio):
    """(color int32[n], rounds): Jones-Plassmann rounds (see orc_color_jp)."""
    n = len(row_ptr) - 1
    c = np.empty(max(n, 1), dtype=np.int32)
    k = _load().orc_color_jp(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(prio, np.uint32), c)
    if k < 0:
        raise MemoryError("orc_color_jp")
    return c[:n], int(k)


def color_certify(row_ptr, col, prio, color):
    """(violations, first_violating_vertex) of the recurrence that fixes the coloring."""
    n = len(row_ptr) - 1
    first = ctypes.c_int64(-1)
    bad = _load().orc_color_certify(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(prio, np.uint32),
                                    _nonempty(color, np.int32), ctypes.byref(first))
    return int(bad), int(first.value)


def spmv_f64(row_ptr, col, val, x):
    """(y_ref, b): binary64 product and per-row sum of |a_ij x_j|."""
    n = len(row_ptr) - 1
    y = np.empty(max(n, 1), dtype=np.float64)
    b = np.empty(max(n, 1), dtype=np.float64)
    _load().orc_spmv_f64(n, _i32(row_ptr), _nonempty(col, np.int32), _nonempty(val, np.float32),
                         _nonempty(x, np.float32), y, b)
    return y[:n], b[:n]


def spmv_f64_threads(row_ptr, col, val, x, threads: int):
    """spmv_f64 with the rows split into `threads` blocks of about equal nonzero
    counts, each block computed by orc_spmv_f64 on its own host thread (the
    arithmetic of every row is that of spmv_f64; only the rows run side by
    side).  For timing the oracle on all host cores."""
    import concurrent.futures as cf
    n = len(row_ptr) - 1
    rp = _i32(row_ptr)
    c, v, xx = _nonempty(col, np.int32), _nonempty(val, np.float32), _nonempty(x, np.float32)
    y = np.empty(max(n, 1), dtype=np.float64)
    b = np.empty(max(n, 1), dtype=np.float64)
    m = int(rp[n]) if n > 0 else 0
    cuts = [0] + [int(np.searchsorted(rp, m * k // threads, side="left")) for k in range(1, threads)] + [n]
    cuts = sorted(set(min(max(q, 0), n) for q in cuts))
    lib = _load()

    def block(lo, hi):
        if hi > lo:
            lib.orc_spmv_f64(hi - lo, rp[lo:hi + 1], c, v, xx, y[lo:hi], b[lo:hi])

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda p: block(*p), zip(cuts[:-1], cuts[1:])))
    return y[:n], b[:n]


SPMV_RTOL = 1e-5


def pagerank_f64(in_row_ptr, in_col, out_degree, iterations: int, damping: float = 0.85):
    """Binary64 PageRank after `iterations` sweeps from 1/n (see orc_pagerank_f64)."""
    n = len(in_row_ptr) - 1
    r = np.empty(max(n, 1), dtype=np.float64)
    if _load().orc_pagerank_f64(n, _i32(in_row_ptr), _nonempty(in_col, np.int32), _nonempty(out_degree, np.int32),
                                int(iterations), float(damping), r) != 0:
        raise MemoryError("orc_pagerank_f64")
    return r[:n]


# Default relative bound of fp32 ranks against the binary64 oracle (all ranks
# are at least (1 - d) / n > 0, so a relative bound is meaningful).  All terms
# are positive, so a sweep whose sums round no term more than D times adds at
# most gamma(D + 5) = (D + 5) u / (1 - (D + 5) u), u = 2^-24, to the relative
# error it inherits (the inherited error is not damped at a hub, where the
# damped sum dominates the constant term): K sweeps stay within
# (1 + u)(1 + gamma(D + 5))^K - 1, which is below 1e-4 for K <= 10 and
# D <= 160.  The parity tests derive the bound for each mode, tune and K from
# the depth of the kernels' sums and pass it as rtol.
PAGERANK_RTOL = 1e-4


def pagerank_check(r_ref, r, rtol: float = PAGERANK_RTOL):
    """(bad_vertices, first_bad_vertex) for |r - r_ref| <= rtol * r_ref."""
    r = np.asarray(r, dtype=np.float64)
    bad = np.flatnonzero(~(np.abs(r - r_ref) <= rtol * r_ref))
    return int(bad.size), int(bad[0]) if bad.size else -1


def spmv_check(y_ref, b, y, rtol: float = SPMV_RTOL):
    """(bad_rows, first_bad_row) for the per-row test |y - y_ref| <= rtol * b."""
    n = len(y_ref)
    first = ctypes.c_int64(-1)
    bad = _load().orc_spmv_check(n, _nonempty(y_ref, np.float64), _nonempty(b, np.float64),
                                 _nonempty(y, np.float32), rtol, ctypes.byref(first))
    return int(bad), first.value


# ---- trees --------------------------------------------------------------------------------------

def tree_validate(parent, child_ptr, child) -> int:
    n = len(parent)
    return _load().orc_tree_validate(n, _i32(parent), _i32(child_ptr), _nonempty(child, np.int32))


def tree_descendants(child_ptr, child) -> np.ndarray:
    n = len(child_ptr) - 1
    out = np.empty(n, dtype=np.int32)
    rc = _load().orc_tree_descendants(n, _i32(child_ptr), _nonempty(child, np.int32), out)
    if rc != 0:
        raise ValueError(f"orc_tree_descendants failed ({rc})")
    return out


def tree_height(child_ptr, child) -> np.ndarray:
    n = len(child_ptr) - 1
    out = np.empty(n, dtype=np.int32)
    rc = _load().orc_tree_height(n, _i32(child_ptr), _nonempty(child, np.int32), out)
    if rc != 0:
        raise ValueError(f"orc_tree_height failed ({rc})")
    return out


def tree_descendants_brute(parent) -> np.ndarray:
    n = len(parent)
    out = np.empty(n, dtype=np.int32)
    if _load().orc_tree_descendants_brute(n, _i32(parent), out) != 0:
        raise ValueError("parent array has a cycle")
    return out


def tree_height_brute(parent) -> np.ndarray:
    n = len(parent)
    out = np.empty(n, dtype=np.int32)
    if _load().orc_tree_height_brute(n, _i32(parent), out) != 0:
        raise ValueError("parent array has a cycle")
    return out


# ---- consolidation bookkeeping ------------------------------------------------------------------

def count_heavy(work, threshold: int) -> int:
    work = np.ascontiguousarray(work, dtype=np.int64)
    return int(_load().orc_count_heavy(len(work), _nonempty(work, np.int64), threshold))


def consolidation_plan(work, threshold: int, scope: int) -> dict:
    work = np.ascontiguousarray(work, dtype=np.int64)
    out = [ctypes.c_int64() for _ in range(4)]
    _load().orc_consolidation_plan(len(work), _nonempty(work, np.int64), threshold, scope,
                                   *[ctypes.byref(o) for o in out])
    return dict(basic_launches=out[0].value, dispatches=out[1].value, items=out[2].value, total_work=out[3].value)


def per_buffer_size(total_thread: int, total_buff_var: int, items_per_thread: int = 4) -> int:
    return int(_load().orc_per_buffer_size(total_thread, total_buff_var, items_per_thread))


def kc_config(blocks: int, threads: int, x: int):
    b, t = ctypes.c_int64(), ctypes.c_int64()
    _load().orc_kc_config(blocks, threads, x, ctypes.byref(b), ctypes.byref(t))
    return b.value, t.value
