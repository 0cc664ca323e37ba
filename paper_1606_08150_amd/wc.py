"""ctypes binding of libwc.so (include/wc.h).  Argument marshalling only: every
step of every problem runs in the library's HIP kernels.  PyTorch provides the
device memory (tensors) and the stream.

The binding refuses to run without the built library or without a GPU; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwc.so")

FLAT, WAVE, BLOCK, GRID = 0, 1, 2, 3
MODES = {"flat": FLAT, "wave": WAVE, "block": BLOCK, "grid": GRID}
STATUS = {0: "WC_OK", -1: "WC_EINVAL", -2: "WC_ENOMEM", -3: "WC_EOVERFLOW", -4: "WC_ETIMEOUT", -5: "WC_EHIP",
          1: "WC_PLANNED"}

# C-ABI symbols declared in include/wc.h
EXPORTS = ("wc_ctx_create", "wc_ctx_destroy", "wc_sssp", "wc_bfs", "wc_spmv", "wc_spmv_noalloc", "wc_spmv_prepare",
           "wc_spmv_hot", "wc_pagerank",
           "wc_color", "wc_tree_descendants", "wc_tree_height", "wc_tree_descendants_batch", "wc_tree_height_batch",
           "wc_sssp_batch", "wc_ctx_set_timing", "wc_ctx_set_wait_limit", "wc_ctx_set_plan_only",
           "wc_ctx_planned_bytes", "wc_ctx_pool_info", "wc_ctx_reserve", "wc_ctx_kernel_stats",
           "wc_ctx_kernel_record", "wc_last_error", "wc_version", "wc_per_buffer_size", "wc_kc_config",
           "wc_default_tune")


class WcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p)]


class CTree(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("parent", ctypes.c_void_p), ("child_ptr", ctypes.c_void_p),
                ("child", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("items_per_lane", ctypes.c_int32), ("driver", ctypes.c_int32), ("allow_fallback", ctypes.c_int32),
                ("buf_capacity", ctypes.c_int64), ("buffer_alloc", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("overflowed", ctypes.c_int32), ("items_buffered", ctypes.c_int64),
                ("dispatches", ctypes.c_int64), ("edges_processed", ctypes.c_int64),
                ("edges_buffered", ctypes.c_int64), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("updates", ctypes.c_int64), ("updates_buffered", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load libwc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1606_08150_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp = c.c_void_p
    lib.wc_ctx_create.restype = c.c_int
    lib.wc_ctx_create.argtypes = [c.c_int, c.c_size_t, c.POINTER(vp)]
    lib.wc_ctx_destroy.restype = c.c_int
    lib.wc_ctx_destroy.argtypes = [vp]
    lib.wc_sssp.restype = c.c_int
    lib.wc_sssp.argtypes = [vp, c.POINTER(CCsr), vp, c.c_int32, vp, c.c_int, c.POINTER(Tune), vp, c.POINTER(Stats)]
    lib.wc_bfs.restype = c.c_int
    lib.wc_bfs.argtypes = [vp, c.POINTER(CCsr), c.c_int32, vp, c.c_int, c.POINTER(Tune), vp, c.POINTER(Stats)]
    lib.wc_spmv.restype = c.c_int
    lib.wc_spmv.argtypes = [vp, c.POINTER(CCsr), vp, vp, vp, c.c_int, c.POINTER(Tune), vp, c.POINTER(Stats)]
    lib.wc_spmv_noalloc.restype = c.c_int
    lib.wc_spmv_noalloc.argtypes = [c.POINTER(CCsr), vp, vp, vp, c.c_int, c.POINTER(Tune), vp]
    lib.wc_spmv_prepare.restype = c.c_int
    lib.wc_spmv_prepare.argtypes = [vp, c.POINTER(CCsr), c.c_int32, vp, vp, vp]
    lib.wc_spmv_hot.restype = c.c_int
    lib.wc_spmv_hot.argtypes = [vp, c.POINTER(CCsr), c.c_int32, vp, vp, vp, vp, c.c_int, c.POINTER(Tune), vp,
                                c.POINTER(Stats)]
    lib.wc_color.restype = c.c_int
    lib.wc_color.argtypes = [vp, c.POINTER(CCsr), vp, vp, c.c_int, c.POINTER(Tune), vp, c.POINTER(Stats)]
    lib.wc_pagerank.restype = c.c_int
    lib.wc_pagerank.argtypes = [vp, c.POINTER(CCsr), vp, c.c_int32, c.c_float, vp, c.c_int, c.POINTER(Tune), vp,
                                c.POINTER(Stats)]
    for name in ("wc_tree_descendants", "wc_tree_height"):
        fn = getattr(lib, name)
        fn.restype = c.c_int
        fn.argtypes = [vp, c.POINTER(CTree), vp, c.c_int, c.POINTER(Tune), vp, c.POINTER(Stats)]
    for name in ("wc_tree_descendants_batch", "wc_tree_height_batch"):
        fn = getattr(lib, name)
        fn.restype = c.c_int
        fn.argtypes = [vp, c.c_int32, c.POINTER(CTree), c.POINTER(vp), c.c_int, c.POINTER(Tune), vp,
                       c.POINTER(Stats)]
    lib.wc_sssp_batch.restype = c.c_int
    lib.wc_sssp_batch.argtypes = [vp, c.c_int32, c.POINTER(CCsr), c.POINTER(vp), c.POINTER(c.c_int32), c.POINTER(vp),
                                  c.POINTER(c.c_int), c.POINTER(Tune), c.c_int32, vp, c.POINTER(Stats)]
    lib.wc_ctx_set_timing.restype = c.c_int
    lib.wc_ctx_set_timing.argtypes = [vp, c.c_int]
    lib.wc_ctx_set_plan_only.restype = c.c_int
    lib.wc_ctx_set_plan_only.argtypes = [vp, c.c_int]
    lib.wc_ctx_planned_bytes.restype = c.c_int
    lib.wc_ctx_planned_bytes.argtypes = [vp, c.POINTER(c.c_size_t)]
    lib.wc_ctx_pool_info.restype = c.c_int
    lib.wc_ctx_pool_info.argtypes = [vp, c.POINTER(c.c_size_t), c.POINTER(c.c_int64)]
    lib.wc_ctx_reserve.restype = c.c_int
    lib.wc_ctx_reserve.argtypes = [vp, c.c_size_t]
    lib.wc_ctx_set_wait_limit.restype = c.c_int
    lib.wc_ctx_set_wait_limit.argtypes = [vp, c.c_int64]
    lib.wc_ctx_kernel_stats.restype = c.c_int
    lib.wc_ctx_kernel_stats.argtypes = [vp, c.c_int32, c.POINTER(c.c_char_p), c.POINTER(c.c_int64),
                                        c.POINTER(c.c_double), c.POINTER(c.c_double)]
    lib.wc_ctx_kernel_record.restype = c.c_int
    lib.wc_ctx_kernel_record.argtypes = [vp, c.c_int32, c.POINTER(c.c_char_p), c.POINTER(c.c_double)]
    lib.wc_last_error.restype = c.c_char_p
    lib.wc_last_error.argtypes = []
    lib.wc_version.restype = c.c_char_p
    lib.wc_per_buffer_size.restype = c.c_int64
    lib.wc_per_buffer_size.argtypes = [c.c_int64, c.c_int64, c.c_int64]
    lib.wc_kc_config.restype = None
    lib.wc_kc_config.argtypes = [c.c_int64, c.c_int64, c.c_int64, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.wc_default_tune.restype = c.c_int
    lib.wc_default_tune.argtypes = [c.c_char_p, c.c_int, c.c_int32, c.POINTER(Tune)]
    _lib = lib
    return lib


def _check(status: int):
    # WC_PLANNED (1): a plan-only context recorded the call's workspace
    if status != 0 and status != 1:
        raise WcError(status, load_library().wc_last_error().decode())


def _mode(mode) -> int:
    if isinstance(mode, str):
        return MODES[mode]
    return int(mode)


def make_tune(**kw) -> Tune:
    t = Tune()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


# ---- host-side planning helpers (no GPU needed) ----------------------------------------------

def per_buffer_size(total_thread: int, total_buff_var: int, items_per_thread: int = 4) -> int:
    return int(load_library().wc_per_buffer_size(total_thread, total_buff_var, items_per_thread))


def kc_config(blocks: int, threads: int, x: int):
    b, t = ctypes.c_int64(), ctypes.c_int64()
    load_library().wc_kc_config(blocks, threads, x, ctypes.byref(b), ctypes.byref(t))
    return b.value, t.value


def default_tune(problem: str, mode, resident_blocks: int) -> dict:
    t = Tune()
    _check(load_library().wc_default_tune(problem.encode(), _mode(mode), resident_blocks, ctypes.byref(t)))
    return t.as_dict()


# ---- device data --------------------------------------------------------------------------------

@dataclass
class DeviceCSR:
    n: int
    row_ptr: torch.Tensor  # int32[n+1]
    col: torch.Tensor      # int32[m]

    @property
    def m(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_host(row_ptr, col, device="cuda"):
        rp = torch.as_tensor(row_ptr, dtype=torch.int32).to(device)
        cl = torch.as_tensor(col, dtype=torch.int32).to(device)
        return DeviceCSR(int(rp.numel()) - 1, rp, cl)

    def c(self) -> CCsr:
        return CCsr(self.n, self.m, self.row_ptr.data_ptr(), self.col.data_ptr() if self.m else None)


@dataclass
class DeviceTree:
    n: int
    parent: torch.Tensor
    child_ptr: torch.Tensor
    child: torch.Tensor

    @staticmethod
    def from_host(parent, child_ptr, child, device="cuda"):
        p = torch.as_tensor(parent, dtype=torch.int32).to(device)
        cp = torch.as_tensor(child_ptr, dtype=torch.int32).to(device)
        ch = torch.as_tensor(child, dtype=torch.int32).to(device)
        return DeviceTree(int(p.numel()), p, cp, ch)

    def c(self) -> CTree:
        return CTree(self.n, self.parent.data_ptr(), self.child_ptr.data_ptr(),
                     self.child.data_ptr() if self.child.numel() else None)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def spmv_noalloc(a: DeviceCSR, val: torch.Tensor, x: torch.Tensor, out: torch.Tensor, mode="grid",
                 tune: Tune | None = None, stream=None) -> torch.Tensor:
    """y = A x through wc_spmv_noalloc (no context, no device allocation in the
    call): `out` (fp32[n], device) is written and returned.  Runs on the current
    device; the caller synchronizes."""
    ca = a.c()
    _check(load_library().wc_spmv_noalloc(ctypes.byref(ca), val.data_ptr() if a.m else None, x.data_ptr(),
                                          out.data_ptr(), _mode(mode), ctypes.byref(tune) if tune else None,
                                          _stream_ptr(stream)))
    return out


class Context:
    """A libwc context: one device pool (the pre-allocated allocator) per device."""

    def __init__(self, device: int = 0, pool_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libwc needs a HIP GPU; none is visible")
        lib = load_library()
        torch.cuda.set_device(device)
        self.device = device
        self._ptr = ctypes.c_void_p()
        _check(lib.wc_ctx_create(device, pool_bytes, ctypes.byref(self._ptr)))

    def close(self):
        if self._ptr:
            load_library().wc_ctx_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- per-kernel timing --
    def set_timing(self, enable: bool):
        _check(load_library().wc_ctx_set_timing(self._ptr, 1 if enable else 0))

    def workspace_bytes(self, fn) -> int:
        """Pool bytes the calls made by fn(self) would carve (plan-only mode:
        nothing is enqueued; results of those calls are not computed)."""
        lib = load_library()
        _check(lib.wc_ctx_set_plan_only(self._ptr, 1))
        try:
            fn(self)
            b = ctypes.c_size_t()
            _check(lib.wc_ctx_planned_bytes(self._ptr, ctypes.byref(b)))
            return int(b.value)
        finally:
            lib.wc_ctx_set_plan_only(self._ptr, 0)

    def pool_info(self):
        """(pool bytes, number of times the pool has grown)."""
        b, g = ctypes.c_size_t(), ctypes.c_int64()
        _check(load_library().wc_ctx_pool_info(self._ptr, ctypes.byref(b), ctypes.byref(g)))
        return int(b.value), int(g.value)

    def reserve(self, nbytes: int):
        """Grow the pool to at least nbytes now (waits for the device)."""
        _check(load_library().wc_ctx_reserve(self._ptr, int(nbytes)))

    def set_wait_limit(self, microseconds: int):
        """Bound of the device-side waits of later calls (<= 0: the default 2 s)."""
        _check(load_library().wc_ctx_set_wait_limit(self._ptr, int(microseconds)))

    def kernel_times(self) -> dict:
        """{kernel name: (launches, total_ms, max_ms)} for the launches recorded
        since timing was enabled."""
        lib = load_library()
        out = {}
        i = 0
        while True:
            name, n = ctypes.c_char_p(), ctypes.c_int64()
            tot, mx = ctypes.c_double(), ctypes.c_double()
            st = lib.wc_ctx_kernel_stats(self._ptr, i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(tot),
                                         ctypes.byref(mx))
            if st != 0:
                break
            out[name.value.decode()] = (n.value, tot.value, mx.value)
            i += 1
        return out

    def kernel_records(self) -> list:
        """[(kernel name, ms)] for every recorded launch, in launch order."""
        lib = load_library()
        out = []
        i = 0
        while True:
            name, ms = ctypes.c_char_p(), ctypes.c_double()
            if lib.wc_ctx_kernel_record(self._ptr, i, ctypes.byref(name), ctypes.byref(ms)) != 0:
                break
            out.append((name.value.decode(), ms.value))
            i += 1
        return out

    # -- problems --
    def sssp(self, g: DeviceCSR, w: torch.Tensor, src: int, mode="grid", tune: Tune | None = None,
             out: torch.Tensor | None = None, stream=None, stats: bool = False):
        dist = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        st = Stats() if stats else None
        cg = g.c()
        _check(load_library().wc_sssp(self._ptr, ctypes.byref(cg), w.data_ptr() if g.m else None, src,
                                      dist.data_ptr(), _mode(mode), ctypes.byref(tune) if tune else None,
                                      _stream_ptr(stream), ctypes.byref(st) if st else None))
        return (dist, st.as_dict()) if stats else dist

    def sssp_batch(self, graphs, weights, sources, modes=None, tunes=None, outs=None, graph_rounds: int = 0,
                   stream=None, stats: bool = False):
        """Batched SSSP over independent instances (lists of DeviceCSR, weight
        tensors, source ints; optional per-instance modes and Tune structs)."""
        k = len(graphs)
        outs = outs if outs is not None else [torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
                                              for g in graphs]
        cg = (CCsr * k)(*[g.c() for g in graphs])
        vp = ctypes.c_void_p
        cw = (vp * k)(*[w.data_ptr() if g.m else None for g, w in zip(graphs, weights)])
        cs = (ctypes.c_int32 * k)(*[int(s) for s in sources])
        cd = (vp * k)(*[o.data_ptr() for o in outs])
        cm = (ctypes.c_int * k)(*[_mode(m) for m in modes]) if modes is not None else None
        ct = (Tune * k)(*tunes) if tunes is not None else None
        st = Stats() if stats else None
        _check(load_library().wc_sssp_batch(self._ptr, k, cg, cw, cs, cd, cm, ct, graph_rounds, _stream_ptr(stream),
                                            ctypes.byref(st) if st else None))
        return (outs, st.as_dict()) if stats else outs

    def bfs(self, g: DeviceCSR, src: int, mode="grid", tune: Tune | None = None, out: torch.Tensor | None = None,
            stream=None, stats: bool = False):
        """Breadth-first levels from src (int32 view of uint32; -1 = unreachable)."""
        lv = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        st = Stats() if stats else None
        cg = g.c()
        _check(load_library().wc_bfs(self._ptr, ctypes.byref(cg), int(src), lv.data_ptr(), _mode(mode),
                                     ctypes.byref(tune) if tune else None, _stream_ptr(stream),
                                     ctypes.byref(st) if st else None))
        return (lv, st.as_dict()) if stats else lv

    def spmv(self, a: DeviceCSR, val: torch.Tensor, x: torch.Tensor, mode="grid", tune: Tune | None = None,
             out: torch.Tensor | None = None, stream=None, stats: bool = False):
        y = out if out is not None else torch.empty(a.n, dtype=torch.float32, device=a.row_ptr.device)
        st = Stats() if stats else None
        ca = a.c()
        _check(load_library().wc_spmv(self._ptr, ctypes.byref(ca), val.data_ptr() if a.m else None, x.data_ptr(),
                                      y.data_ptr(), _mode(mode), ctypes.byref(tune) if tune else None,
                                      _stream_ptr(stream), ctypes.byref(st) if st else None))
        return (y, st.as_dict()) if stats else y

    def spmv_prepare(self, a: DeviceCSR, hot: int, stream=None):
        """Hot-column layout of a: (DeviceCSR with the remapped columns, hot_ids tensor)."""
        col_hot = torch.empty(max(a.m, 1), dtype=torch.int32, device=a.row_ptr.device)
        hot_ids = torch.empty(max(hot, 1), dtype=torch.int32, device=a.row_ptr.device)
        ca = a.c()
        _check(load_library().wc_spmv_prepare(self._ptr, ctypes.byref(ca), int(hot), col_hot.data_ptr(),
                                              hot_ids.data_ptr(), _stream_ptr(stream)))
        return DeviceCSR(a.n, a.row_ptr, col_hot[:a.m]), hot_ids[:hot]

    def spmv_hot(self, a_hot: DeviceCSR, hot_ids: torch.Tensor, val: torch.Tensor, x: torch.Tensor, mode="grid",
                 tune: Tune | None = None, out: torch.Tensor | None = None, stream=None, stats: bool = False):
        """y = A x in the hot-column layout from spmv_prepare."""
        y = out if out is not None else torch.empty(a_hot.n, dtype=torch.float32, device=a_hot.row_ptr.device)
        st = Stats() if stats else None
        ca = a_hot.c()
        hot = int(hot_ids.numel())
        _check(load_library().wc_spmv_hot(self._ptr, ctypes.byref(ca), hot, hot_ids.data_ptr() if hot else None,
                                          val.data_ptr() if a_hot.m else None, x.data_ptr(), y.data_ptr(),
                                          _mode(mode), ctypes.byref(tune) if tune else None, _stream_ptr(stream),
                                          ctypes.byref(st) if st else None))
        return (y, st.as_dict()) if stats else y

    def pagerank(self, in_graph: DeviceCSR, out_degree: torch.Tensor, iterations: int, damping: float = 0.85,
                 mode="grid", tune: Tune | None = None, out: torch.Tensor | None = None, stream=None,
                 stats: bool = False):
        """Ranks after `iterations` sweeps; in_graph is the transpose (in-edges) of
        the graph, out_degree its vertices' out-degrees (int32, device)."""
        r = out if out is not None else torch.empty(in_graph.n, dtype=torch.float32, device=in_graph.row_ptr.device)
        st = Stats() if stats else None
        cg = in_graph.c()
        _check(load_library().wc_pagerank(self._ptr, ctypes.byref(cg), out_degree.data_ptr(), int(iterations),
                                          float(damping), r.data_ptr(), _mode(mode),
                                          ctypes.byref(tune) if tune else None, _stream_ptr(stream),
                                          ctypes.byref(st) if st else None))
        return (r, st.as_dict()) if stats else r

    def color(self, g: DeviceCSR, prio: torch.Tensor, mode="grid", tune: Tune | None = None,
              out: torch.Tensor | None = None, stream=None, stats: bool = False):
        """Jones-Plassmann colors of a symmetric graph (int32); prio holds the
        vertices' priorities (uint32 values in an int32 or int64 tensor, device)."""
        if prio.dtype not in (torch.int32, torch.uint32) or prio.numel() != g.n:
            raise ValueError("prio must hold n 32-bit priorities")
        c = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
        st = Stats() if stats else None
        cg = g.c()
        _check(load_library().wc_color(self._ptr, ctypes.byref(cg), prio.data_ptr(), c.data_ptr(), _mode(mode),
                                       ctypes.byref(tune) if tune else None, _stream_ptr(stream),
                                       ctypes.byref(st) if st else None))
        return (c, st.as_dict()) if stats else c

    def _tree(self, fn, t: DeviceTree, mode, tune, out, stream, stats):
        res = out if out is not None else torch.empty(t.n, dtype=torch.int32, device=t.parent.device)
        st = Stats() if stats else None
        ct = t.c()
        _check(fn(self._ptr, ctypes.byref(ct), res.data_ptr(), _mode(mode), ctypes.byref(tune) if tune else None,
                  _stream_ptr(stream), ctypes.byref(st) if st else None))
        return (res, st.as_dict()) if stats else res

    def tree_descendants(self, t: DeviceTree, mode="grid", tune: Tune | None = None, out=None, stream=None,
                         stats: bool = False):
        return self._tree(load_library().wc_tree_descendants, t, mode, tune, out, stream, stats)

    def tree_height(self, t: DeviceTree, mode="grid", tune: Tune | None = None, out=None, stream=None,
                    stats: bool = False):
        return self._tree(load_library().wc_tree_height, t, mode, tune, out, stream, stats)

    def _tree_batch(self, fn, trees, mode, tune, outs, stream, stats):
        k = len(trees)
        outs = outs if outs is not None else [torch.empty(t.n, dtype=torch.int32, device=t.parent.device)
                                              for t in trees]
        ct = (CTree * k)(*[t.c() for t in trees])
        co = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
        st = Stats() if stats else None
        _check(fn(self._ptr, k, ct, co, _mode(mode), ctypes.byref(tune) if tune else None, _stream_ptr(stream),
                  ctypes.byref(st) if st else None))
        return (outs, st.as_dict()) if stats else outs

    def tree_descendants_batch(self, trees, mode="grid", tune: Tune | None = None, outs=None, stream=None,
                               stats: bool = False):
        """Descendant counts of every tree of a list of DeviceTrees, in one call."""
        return self._tree_batch(load_library().wc_tree_descendants_batch, trees, mode, tune, outs, stream, stats)

    def tree_height_batch(self, trees, mode="grid", tune: Tune | None = None, outs=None, stream=None,
                          stats: bool = False):
        """Heights of every tree of a list of DeviceTrees, in one call."""
        return self._tree_batch(load_library().wc_tree_height_batch, trees, mode, tune, outs, stream, stats)
