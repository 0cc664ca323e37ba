"""Seeded synthetic inputs shared by the oracle and the GPU path.

The generators live in ``synth.c`` (built into ``libsynth.so`` by
``synth.build.build()``); this module only marshals numpy arrays.  Nothing in
here computes any part of the consolidation method: it produces graphs, trees,
weights, values and vectors, and the small hand-built shapes the tests use.

Seeds follow one convention everywhere: 1 graph structure, 2 edge weights,
3 matrix values, 4 the dense vector x, 5 trees.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

SEED_GRAPH, SEED_WEIGHT, SEED_VALUE, SEED_X, SEED_TREE = 1, 2, 3, 4, 5
RMAT_ABC = (0.57, 0.19, 0.19)  # d = 0.05


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing; run synth.build.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    c = ctypes
    lib.syn_rand.restype = c.c_uint64
    lib.syn_rand.argtypes = [c.c_uint64, c.c_uint64, c.c_uint64]
    lib.syn_rand_fill.restype = None
    lib.syn_rand_fill.argtypes = [c.c_uint64, c.c_uint64, c.c_int64, u64p]
    lib.syn_rmat_edges.restype = c.c_int
    lib.syn_rmat_edges.argtypes = [c.c_int, c.c_int64, c.c_uint64, c.c_double, c.c_double, c.c_double, i32p, i32p]
    lib.syn_rmat_edges_n.restype = c.c_int
    lib.syn_rmat_edges_n.argtypes = [c.c_int64, c.c_int64, c.c_uint64, c.c_double, c.c_double, c.c_double, i32p, i32p]
    lib.syn_csr_from_edges.restype = c.c_int
    lib.syn_csr_from_edges.argtypes = [c.c_int64, c.c_int64, i32p, i32p, i32p, i32p]
    lib.syn_weights.restype = None
    lib.syn_weights.argtypes = [c.c_int64, c.c_uint64, c.c_uint32, u32p]
    lib.syn_uniform_pm1.restype = None
    lib.syn_uniform_pm1.argtypes = [c.c_int64, c.c_uint64, c.c_uint64, f32p]
    lib.syn_random_tree.restype = c.c_int
    lib.syn_random_tree.argtypes = [c.c_int64, c.c_uint64, c.c_int32, c.c_double, c.c_int32, i32p, i32p, i32p,
                                    c.c_void_p]
    _lib = lib
    return lib


@dataclass
class CSR:
    """Directed graph / sparse matrix in CSR form: row = source vertex."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[m]

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


@dataclass
class Tree:
    """Rooted tree, root 0: parent[n] (parent[0] = -1), child CSR child_ptr[n+1], child[n-1]."""

    n: int
    parent: np.ndarray
    child_ptr: np.ndarray
    child: np.ndarray
    depth: np.ndarray | None = None


def rand_u64(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().syn_rand_fill(seed, stream, count, out)
    return out


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(m, dtype=np.int32)
    rc = _load().syn_csr_from_edges(n, m, src, dst, row_ptr, col)
    if rc != 0:
        raise ValueError(f"csr_from_edges failed ({rc})")
    return CSR(n, row_ptr, col)


def rmat_edges(scale: int, m: int, seed: int = SEED_GRAPH, abc=RMAT_ABC):
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().syn_rmat_edges(scale, m, seed, abc[0], abc[1], abc[2], src, dst)
    if rc != 0:
        raise ValueError(f"rmat_edges failed ({rc})")
    return src, dst


def rmat_csr(scale: int, m: int, seed: int = SEED_GRAPH, abc=RMAT_ABC) -> CSR:
    """R-MAT graph on 2^scale vertices with exactly m directed edges."""
    src, dst = rmat_edges(scale, m, seed, abc)
    return csr_from_edges(1 << scale, src, dst)


def rmat_csr_n(n: int, m: int, seed: int, abc=RMAT_ABC) -> CSR:
    """R-MAT graph on n vertices (any n >= 1): pairs outside [0, n) are rejected."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().syn_rmat_edges_n(n, m, seed, abc[0], abc[1], abc[2], src, dst)
    if rc != 0:
        raise ValueError(f"rmat_edges_n failed ({rc})")
    return csr_from_edges(n, src, dst)


def weights(m: int, seed: int = SEED_WEIGHT, wmax: int = 100) -> np.ndarray:
    """uint32 edge weights uniform on 1..wmax, indexed by CSR position."""
    w = np.empty(m, dtype=np.uint32)
    _load().syn_weights(m, seed, wmax, w)
    return w


def uniform_pm1(count: int, seed: int, stream: int = 0) -> np.ndarray:
    """float32 values uniform in [-1, 1) on the 2^-23 grid."""
    out = np.empty(count, dtype=np.float32)
    _load().syn_uniform_pm1(count, seed, stream, out)
    return out


def values(m: int, seed: int = SEED_VALUE) -> np.ndarray:
    return uniform_pm1(m, seed, 0)


def vector_x(n: int, seed: int = SEED_X, stream: int = 0) -> np.ndarray:
    return uniform_pm1(n, seed, stream)


def random_tree(n: int, seed: int = SEED_TREE, kmax: int = 4096, alpha: float = 2.0, max_depth: int = 24,
                with_depth: bool = False) -> Tree:
    """Random rooted tree with truncated power-law fanout (see synth.c)."""
    parent = np.empty(n, dtype=np.int32)
    child_ptr = np.empty(n + 1, dtype=np.int32)
    child = np.empty(max(n - 1, 0), dtype=np.int32)
    depth = np.empty(n, dtype=np.int32) if with_depth else None
    dptr = depth.ctypes.data_as(ctypes.c_void_p) if depth is not None else None
    rc = _load().syn_random_tree(n, seed, kmax, alpha, max_depth, parent, child_ptr,
                                 child if n > 1 else np.empty(1, np.int32), dptr)
    if rc != 0:
        raise ValueError(f"random_tree failed ({rc})")
    return Tree(n, parent, child_ptr, child, depth)


def layered_tree(levels: int, fan_lo: int, fan_hi: int, internal_fraction: float = 1.0, seed: int = SEED_TREE,
                 stream: int = 500) -> Tree:
    """Tree of fixed depth in the manner of the paper's tree sets (Sec. V):
    every node above the last level has children with probability
    internal_fraction (the root always), and then a fanout drawn uniformly from
    [fan_lo, fan_hi]; nodes are numbered level by level, a node's children
    consecutively.  Level d's draws come from streams (stream + 2d, stream + 2d + 1)."""
    if not (1 <= fan_lo <= fan_hi) or levels < 0:
        raise ValueError("bad layered tree parameters")
    parent = [np.array([-1], dtype=np.int64)]
    level = np.array([0], dtype=np.int64)
    next_id = 1
    for d in range(levels):
        k = level.size
        r1 = rand_u64(seed, stream + 2 * d, k)
        r2 = rand_u64(seed, stream + 2 * d + 1, k)
        has = (r1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 < internal_fraction
        if d == 0:
            has[:] = True
        fan = np.where(has, fan_lo + (r2 % np.uint64(fan_hi - fan_lo + 1)).astype(np.int64), 0)
        total = int(fan.sum())
        if next_id + total > 2 ** 31 - 1:
            raise ValueError("layered tree larger than int32 ids allow")
        parent.append(np.repeat(level, fan))
        level = np.arange(next_id, next_id + total, dtype=np.int64)
        next_id += total
    return tree_from_parent(np.concatenate(parent).astype(np.int32))


# ---- batches of independent instances ----------------------------------------------------------

def batch_sizes(count: int, lo_log2: float = 10.0, hi_log2: float = 18.0, seed: int = SEED_GRAPH,
                stream: int = 300) -> np.ndarray:
    """Vertex counts log-uniform in [2^lo, 2^hi]: n_i = floor(2^U), U uniform (one draw per instance)."""
    r = rand_u64(seed, stream, count)
    u = (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def batch_instances(count: int, degree: int = 16, lo_log2: float = 10.0, hi_log2: float = 18.0,
                    seed: int = SEED_GRAPH):
    """`count` independent R-MAT instances: instance i has n_i vertices (batch_sizes)
    and degree * n_i edges, drawn at scale ceil(log2 n_i) with out-of-range
    endpoints rejected; graph seed (seed, i) and weight seed (SEED_WEIGHT, i) are
    folded into one 64-bit seed each.  Returns a list of (CSR, weights)."""
    sizes = batch_sizes(count, lo_log2, hi_log2, seed)
    out = []
    for i, n in enumerate(sizes.tolist()):
        gseed = int(_load().syn_rand(seed, 301, i))
        wseed = int(_load().syn_rand(SEED_WEIGHT, 302, i))
        g = rmat_csr_n(int(n), int(degree * n), gseed)
        out.append((g, weights(g.m, wseed)))
    return out


def batch_trees(count: int, lo_log2: float = 4.0, hi_log2: float = 16.0, seed: int = SEED_TREE) -> list:
    """`count` independent random trees (random_tree's generator) with node
    counts log-uniform in [2^lo, 2^hi] (batch_sizes, stream 310); tree i uses the
    64-bit seed folded from (seed, 311, i)."""
    sizes = batch_sizes(count, lo_log2, hi_log2, seed, stream=310)
    return [random_tree(max(1, int(n)), seed=int(_load().syn_rand(seed, 311, i))) for i, n in enumerate(sizes.tolist())]


def serving_graph_sizes(count: int = 64, lo_log2: float = 14.0, hi_log2: float = 20.0) -> list:
    """Vertex counts round(2^(lo + (hi - lo) k / (count - 1))), k = 0..count-1."""
    if count == 1:
        return [int(round(2 ** lo_log2))]
    return [int(round(2 ** (lo_log2 + (hi_log2 - lo_log2) * k / (count - 1)))) for k in range(count)]


def serving_graph(k: int, n: int, degree: int = 16, n_x: int = 4):
    """Resident graph k of the serving workload: R-MAT on n vertices with
    degree * n edges, weights, matrix values and n_x dense vectors, each from
    seeds derived from (kind, k)."""
    gseed = int(_load().syn_rand(SEED_GRAPH, 401, k))
    g = rmat_csr_n(n, degree * n, gseed)
    w = weights(g.m, int(_load().syn_rand(SEED_WEIGHT, 402, k)))
    val = values(g.m, int(_load().syn_rand(SEED_VALUE, 403, k)))
    xs = [vector_x(n, int(_load().syn_rand(SEED_X, 404, k)), stream=j) for j in range(n_x)]
    return g, w, val, xs


# ---- small hand-built shapes (tests and edge cases) -------------------------------------------

def tree_from_parent(parent) -> Tree:
    """Tree from a parent array (parent[0] = -1); child lists sorted by id."""
    parent = np.asarray(parent, dtype=np.int32)
    n = parent.shape[0]
    if n == 0 or parent[0] != -1:
        raise ValueError("parent[0] must be -1")
    counts = np.bincount(parent[1:], minlength=n).astype(np.int64) if n > 1 else np.zeros(1, np.int64)
    child_ptr = np.zeros(n + 1, dtype=np.int64)
    child_ptr[1:] = np.cumsum(counts)
    order = np.lexsort((np.arange(1, n), parent[1:])) if n > 1 else np.empty(0, np.int64)
    child = (np.arange(1, n)[order]).astype(np.int32)
    return Tree(n, parent, child_ptr.astype(np.int32), child)


def chain_tree(n: int) -> Tree:
    return tree_from_parent(np.concatenate([[-1], np.arange(n - 1)]).astype(np.int32))


def star_tree(n: int) -> Tree:
    return tree_from_parent(np.concatenate([[-1], np.zeros(n - 1)]).astype(np.int32))


def kary_tree(k: int, height: int) -> Tree:
    """Complete k-ary tree of the given height (a lone root has height 0)."""
    n = sum(k ** i for i in range(height + 1))
    parent = np.empty(n, dtype=np.int32)
    parent[0] = -1
    parent[1:] = (np.arange(1, n) - 1) // k
    return tree_from_parent(parent)


def transpose(g: CSR) -> CSR:
    """The reversed graph: row v lists the sources u of the edges u -> v, in
    increasing u (multi-edges kept).  A data-layout step for in-edge (pull)
    iterations; holds no arithmetic of the method."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    dst = g.col.astype(np.int64)
    order = np.lexsort((src, dst))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, dst + 1, 1)
    return CSR(n, np.cumsum(row_ptr).astype(np.int32), src[order].astype(np.int32))


def symmetrize(g: CSR) -> CSR:
    """The undirected graph: every edge in both directions, self-loops and
    repeated edges dropped, rows sorted.  A data-layout step; no arithmetic of
    the method."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    dst = g.col.astype(np.int64)
    keep = src != dst
    a = np.concatenate([src[keep], dst[keep]])
    b = np.concatenate([dst[keep], src[keep]])
    key = np.unique(a * n + b)
    a, b = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, a + 1, 1)
    return CSR(n, np.cumsum(row_ptr).astype(np.int32), b.astype(np.int32))


def priorities(n: int, seed: int = SEED_GRAPH, stream: int = 600) -> np.ndarray:
    """Seeded uint32 vertex priorities for the coloring rounds."""
    return (rand_u64(seed, stream, n) >> np.uint64(32)).astype(np.uint32)


def out_degree(g: CSR) -> np.ndarray:
    return np.diff(g.row_ptr).astype(np.int32)


def graph_from_edges(n: int, edges, w=None):
    """Small directed graph from an explicit (u, v) list; returns (CSR, weights) with the
    weights permuted into CSR order."""
    edges = list(edges)
    src = np.array([e[0] for e in edges], dtype=np.int64)
    dst = np.array([e[1] for e in edges], dtype=np.int64)
    wt = np.ones(len(edges), dtype=np.uint32) if w is None else np.asarray(w, dtype=np.uint32)
    order = np.lexsort((dst, src))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    if len(edges):
        np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSR(n, row_ptr.astype(np.int32), dst[order].astype(np.int32)), wt[order]
