/*
 * wc.h - workload consolidation of nested parallel work on AMD MI355X (gfx950).
 *
 * C ABI of libwc.so.  The library implements the consolidation schemes of
 * Wu, Li & Becchi, "Compiler-Assisted Workload Consolidation for Efficient
 * Dynamic Parallelism on GPU" (arXiv 1606.08150), Sec. IV, for the paper's
 * irregular-loop problems (SSSP and SpMV over CSR, Sec. II.B and Fig. 1(b))
 * and parallel-recursion problems (tree descendants and tree heights,
 * Fig. 1(c), Sec. V).
 *
 * gfx950 has no device-side kernel launch, so a consolidated child kernel is
 * an in-kernel drain of a consolidation buffer:
 *   WC_WAVE  - one buffer per 64-lane wavefront, filled with a ballot/prefix
 *              append; no barrier (the wave runs in lockstep, Sec. IV.B).
 *   WC_BLOCK - one buffer per workgroup in LDS; a workgroup barrier separates
 *              the inserts from the drain (Sec. IV.B).
 *   WC_GRID  - one global buffer per grid, filled with wave-aggregated atomic
 *              appends; the whole grid drains it after a grid-wide barrier
 *              (a kernel boundary: the host relaunches one round at a time).
 *   WC_FLAT  - no consolidation: each parent thread does all of its item's
 *              work itself (the paper's flat "no-dp" baseline, Sec. V).
 * All modes compute the same result; the consolidated child processes each
 * buffered item exactly as the unconsolidated work would (Sec. IV.C).
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller; the library never
 *    frees or retains them beyond the call's stream work.
 *  - Work is enqueued on `stream`.  SSSP, BFS, coloring and the trees decide at
 *    run time how many rounds/levels to run: the host waits on device-published
 *    round counts (each tagged with the call's epoch, so a value left by an
 *    earlier call is never taken for this one), and the call returns once the
 *    last round has been enqueued.  The caller synchronizes before reading
 *    outputs, unless `stats` is non-NULL, in which case the call synchronizes
 *    the stream itself to fill it in.
 *  - Device-side waits (the packet queues of the wave and block modes of the
 *    trees) are bounded in time (2 s by default, wc_ctx_set_wait_limit); a call
 *    containing such waits returns only after its kernels are done and reports
 *    WC_ETIMEOUT if a wait gave up, with or without `stats`.
 *  - A context owns one pre-allocated device pool (the custom allocator of
 *    Sec. IV.E) from which every call carves its buffers.  Calls that share a
 *    context must be issued on one stream (or be externally serialized).
 *  - Invalid arguments return WC_EINVAL before anything is enqueued; HIP
 *    failures return WC_EHIP; pool exhaustion that cannot be grown returns
 *    WC_ENOMEM.  wc_last_error() then describes the failure.  No C++
 *    exception crosses this boundary.
 *  - Integer results (distances, descendant counts, heights) are identical in
 *    every mode and launch configuration.  SpMV results are within
 *    |y - y_ref| <= 1e-5 * sum_j |a_ij x_j| per row of the exact product and
 *    are bitwise reproducible for a fixed mode and tune.
 */
#ifndef WC_H
#define WC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Consolidation granularity: the consldt(warp|block|grid) clause of Table I, plus flat. */
typedef enum { WC_FLAT = 0, WC_WAVE = 1, WC_BLOCK = 2, WC_GRID = 3 } wc_mode;

typedef enum {
    WC_OK = 0,
    WC_EINVAL = -1,    /* bad argument; nothing was enqueued */
    WC_ENOMEM = -2,    /* device pool could not be (re)allocated */
    WC_EOVERFLOW = -3, /* a consolidation buffer overflowed and tune->allow_fallback < 0 */
    WC_ETIMEOUT = -4,  /* a bounded device-side or host-side wait expired */
    WC_EHIP = -5,      /* a HIP runtime call failed */
    WC_PLANNED = 1     /* plan-only context (wc_ctx_set_plan_only): the arguments were
                          checked and the call's workspace recorded; nothing was enqueued */
} wc_status;

/* Directed graph / sparse matrix, CSR with row = source vertex.
 * row_ptr[n+1] (row_ptr[0] = 0, row_ptr[n] = m, non-decreasing), col[m] in [0, n). */
typedef struct {
    int32_t n;
    int32_t m;
    const int32_t *row_ptr;
    const int32_t *col;
} wc_csr;

/* Rooted tree, root = node 0.  parent[n] (parent[0] = -1), children in CSR form:
 * child_ptr[n+1] (child_ptr[n] = n-1) and child[n-1]. */
typedef struct {
    int32_t n;
    const int32_t *parent;
    const int32_t *child_ptr;
    const int32_t *child;
} wc_tree;

/* Launch and buffer configuration (the threads/blocks/buffer clauses of Table I
 * and the configuration rules of Sec. IV.E).  A zero (or negative) field means
 * "use the library's heuristic"; pass NULL for all defaults. */
typedef struct {
    int32_t threshold;      /* items with more than this much work are buffered (the
                               THRESHOLD of Fig. 1(b)); <= 0: the default of
                               wc_default_tune (8 for SSSP and SpMV, at grid
                               level except coloring and for coloring at block
                               level; 0 for the trees; 64 for coloring at grid
                               level; 32 otherwise) */
    int32_t block_threads;  /* workgroup size: 64, 128, 256, 512 or 1024; <= 0: the
                               default of wc_default_tune (512 at grid level except
                               coloring; the packet queues: 1024 for BFS and the
                               trees at wave level, 512 for BFS and the trees'
                               descendants at block level; 256 otherwise) */
    int32_t grid_blocks;    /* workgroups of the moldable drain/persistent grid;
                               <= 0: resident maximum from the occupancy query (KC_1).
                               SSSP and SpMV in wave and block modes launch their
                               parent with one workgroup per block_threads items
                               unless this caps it */
    int32_t items_per_lane; /* the "const" of the Sec. IV.E buffer-size estimate: work
                               items per drain lane; grid-level chunks hold
                               64 * items_per_lane elements, queue-mode packets
                               (BFS, trees) about 64 * items_per_lane (wave) or
                               block_threads * items_per_lane (block) children;
                               at most 64; <= 0: the default of wc_default_tune
                               (4; grid level 2, 8 for SpMV; wave and block
                               levels 2 for SSSP and SpMV, 1 for coloring, 32
                               in the queue modes, 64 for BFS at wave level) */
    int32_t driver;         /* 0: one launch per round/level (host relaunch);
                               1: reserved for a persistent co-resident launch: not
                                  available, every entry point refuses it with
                                  WC_EINVAL before enqueueing anything;
                               2: grid mode of SSSP, SpMV and the trees only, for
                                  comparison: basic dynamic parallelism emulated, one
                                  host-launched child per buffered vertex (SSSP), heavy
                                  row (SpMV, one workgroup per row) or internal node
                                  (trees, deepest first; the host reads the tree back),
                                  no consolidation (stats->dispatches counts the child
                                  launches);
                               3: SSSP grid mode only, for comparison: the "1-1 mapping"
                                  configuration of Sec. V.B, the consolidated child
                                  launched with one wave per buffered chunk (the host
                                  reads the buffer size after every parent) */
    int32_t allow_fallback; /* on buffer overflow: >= 0 (default) the item that does not fit
                               is processed inline and stats->overflowed is set;
                               < 0 the call returns WC_EOVERFLOW after its work ends */
    int64_t buf_capacity;   /* grid/queue buffer capacity in entries; <= 0: large enough
                               that no overflow can occur */
    int32_t buffer_alloc;   /* SSSP (and BFS) wave and block modes only, for the allocator
                               comparison of Sec. V.A: where a group's consolidation buffer
                               lives.  0 (default): registers / LDS (the child runs inside the
                               group); 1: a global-memory slice of the context pool per
                               workgroup (the paper's pre-allocated allocator, Sec. IV.E);
                               2: a global-memory buffer from device-side malloc per
                               dispatch, freed after the child (the default allocator).  A
                               failed malloc keeps the items in registers / LDS and sets
                               stats->overflowed.  Any other problem or mode: 0 only. */
    int32_t reserved;       /* 0 */
} wc_tune;

/* Device-side counters of one call (filled when `stats` is non-NULL). */
typedef struct {
    int32_t rounds;          /* SSSP rounds or tree levels executed */
    int32_t overflowed;      /* 1 if any buffer overflowed (items were processed inline) */
    int64_t items_buffered;  /* work items inserted into consolidation buffers */
    int64_t dispatches;      /* consolidated child dispatches (non-empty buffers drained) */
    int64_t edges_processed; /* edges relaxed / nonzeros multiplied / children visited */
    int64_t edges_buffered;  /* the part of edges_processed handled by consolidated children */
    float ms;                /* wall time of the call on its stream, from HIP events */
    int32_t reserved;        /* 0 */
    int64_t updates;         /* SSSP: relaxations that lowered a distance (one atomic min and one
                                frontier stamp each); 0 for the other problems */
    int64_t updates_buffered; /* the part of updates made by consolidated children */
} wc_stats;

typedef struct wc_ctx wc_ctx;

/* Create a context on `device` with a pre-allocated pool of `pool_bytes`
 * (0: 512 MiB).  The pool grows on demand when a call needs more.
 * Returns WC_EINVAL for a bad device or NULL out, WC_EHIP/WC_ENOMEM on failure. */
wc_status wc_ctx_create(int device, size_t pool_bytes, wc_ctx **out);

/* Free the pool and the context.  Waits for the device first.  NULL is a no-op. */
wc_status wc_ctx_destroy(wc_ctx *ctx);

/* Single-source shortest paths (Fig. 1(b)): dist[v] = minimum total weight of a
 * path src -> v over edges with weights w[m] (uint32, >= 1), UINT32_MAX if v is
 * unreachable.  Frontier-driven rounds: every vertex whose distance improved is
 * expanded in the next round; a frontier vertex with more than `threshold`
 * out-edges is consolidated per `mode`, a lighter one relaxes its edges inline.
 * dist[n] is written entirely.  Distances must stay below UINT32_MAX. */
wc_status wc_sssp(wc_ctx *ctx, const wc_csr *g, const uint32_t *w, int32_t src, uint32_t *dist, wc_mode mode,
                  const wc_tune *tune, hipStream_t stream, wc_stats *stats);

/* Breadth-first levels (recursive BFS, the BFS-Rec benchmark of Sec. V): level[v]
 * = number of edges on a shortest path src -> v, UINT32_MAX if v is unreachable.
 * A visit of v is a recursive call whose children are the neighbours it brings
 * to a lower level (parallel recursion, Sec. II.B).
 *   WC_WAVE, WC_BLOCK: the recursion path.  The recursive calls a wave
 *     (workgroup) makes go into its buffer; a full buffer is flushed as
 *     consolidated dispatches, packets of about 64 * items_per_lane (wave) or
 *     block_threads * items_per_lane (block) edges in a device-wide queue that
 *     any group of a persistent grid processes (no grid-wide barrier).  The call of a vertex with more
 *     than 64 * items_per_lane out-edges is split into packets of its own, so
 *     a hub is spread over many groups.  Waits for packets are bounded
 *     (WC_ETIMEOUT).  A call list too small (tune->buf_capacity entries; by
 *     default twice the vertices plus edge chunks) raises stats->overflowed
 *     and the levels are recomputed with the frontier rounds below
 *     (WC_EOVERFLOW instead when tune->allow_fallback < 0).
 *   WC_FLAT, WC_GRID: the calls of one depth (the frontier) are consolidated by
 *     the frontier rounds of wc_sssp with every edge weighing 1, on the same
 *     kernels.
 * level[n] is written entirely.  tune->driver must be 0 in wave and block
 * modes, and tune->buffer_alloc 0. */
wc_status wc_bfs(wc_ctx *ctx, const wc_csr *g, int32_t src, uint32_t *level, wc_mode mode, const wc_tune *tune,
                 hipStream_t stream, wc_stats *stats);

/* Sparse matrix-vector product y = A x, A in CSR with values val[m] (fp32),
 * x[n] and y[n] fp32 (square n x n).  A row with more than `threshold`
 * nonzeros is consolidated per `mode`; a lighter row is summed inline by one
 * lane.  y[n] is written entirely; empty rows give +0. */
wc_status wc_spmv(wc_ctx *ctx, const wc_csr *a, const float *val, const float *x, float *y, wc_mode mode,
                  const wc_tune *tune, hipStream_t stream, wc_stats *stats);

/* Hot-column layout for repeated products with one matrix (a layout choice
 * around the method, not part of it): the x gathers of SpMV go to random
 * columns, and a power-law matrix's most used columns are spread over the
 * whole of x.  wc_spmv_prepare ranks the columns by their number of entries
 * (ties by column id), writes the `hot` most used column ids to hot_ids[hot]
 * (device, most used first) and col_hot[m] (device): col_hot[e] = the rank of
 * col[e] if it is one of the hot columns, else hot + col[e].  Rows, the order
 * of entries and the values are unchanged.  Synchronous (the ranking runs on
 * the host from device-computed counts).  WC_EINVAL for hot outside [0, n],
 * n + hot >= 2^31 or NULL arrays. */
wc_status wc_spmv_prepare(wc_ctx *ctx, const wc_csr *a, int32_t hot, int32_t *col_hot, int32_t *hot_ids,
                          hipStream_t stream);

/* y = A x with A in the hot-column layout (a_hot: the matrix's row_ptr with
 * col_hot as col; hot and hot_ids from wc_spmv_prepare; val and x as for
 * wc_spmv).  The product first gathers the hot columns' x values into a dense
 * array; in grid mode each drain workgroup stages the most used of them in LDS
 * (32 per thread, up to 16384).  Same kernels, mode semantics, tune and
 * summation order as wc_spmv on the original matrix, so results are
 * bit-identical to it. */
wc_status wc_spmv_hot(wc_ctx *ctx, const wc_csr *a_hot, int32_t hot, const int32_t *hot_ids, const float *val,
                      const float *x, float *y, wc_mode mode, const wc_tune *tune, hipStream_t stream,
                      wc_stats *stats);

/* PageRank (the PR benchmark of Sec. V, an irregular loop like SpMV): from
 * rank = 1/n, `iterations` synchronous sweeps of
 *   rank'[v] = (1 - damping) / n + damping * (sum over edges u -> v of rank[u] / outdeg(u) + D / n),
 * D = the rank held by vertices without out-edges (spread over all vertices, so
 * the ranks keep summing to 1).  in_graph holds the in-edges: row v lists the
 * source u of every edge u -> v (the transpose of the out-edge CSR);
 * out_degree[n] (int32, device) is each vertex's number of out-edges.  Each
 * sweep's loop over a vertex's in-edges is consolidated per `mode` exactly as
 * in wc_spmv (unit values).  rank[n] (fp32, device) is written.  fp32 sums in
 * an order fixed by mode and tune: bit-identical across runs for a fixed mode
 * and tune.  stats->rounds = iterations.  WC_EINVAL for negative sizes or
 * iterations, damping outside [0, 1] or NULL arrays. */
wc_status wc_pagerank(wc_ctx *ctx, const wc_csr *in_graph, const int32_t *out_degree, int32_t iterations,
                      float damping, float *rank, wc_mode mode, const wc_tune *tune, hipStream_t stream,
                      wc_stats *stats);

/* Graph coloring (the GC benchmark of Sec. V, an irregular loop): Jones-Plassmann
 * colors of a symmetric graph g (every edge u -> v matched by a v -> u, with the
 * same multiplicity; self-loops are ignored).  Vertex u outranks v when
 * prio[u] > prio[v], or the priorities are equal and u > v.  In round r = 0, 1, ...
 * every uncolored vertex that outranks each of its uncolored neighbours takes
 * color r; equivalently color[v] = 0 if no neighbour outranks v, else 1 + the
 * largest color of an outranking neighbour.  Computed data-driven: a vertex
 * colored in round r releases the neighbours it outranks, and one whose last
 * outranking neighbour that was is colored r + 1; the release loop of a vertex
 * with more than `threshold` neighbours is consolidated per `mode` (wave and
 * block modes hand ranges longer than 64 * items_per_lane on to a grid-wide
 * drain after each pass, as the other irregular loops do).  color[n]
 * (int32, device) is written entirely; prio[n] (uint32, device) is read only.
 * The colors do not depend on mode, tune or schedule.  stats->rounds = number
 * of colors.  Only the relaunch driver exists (tune->driver 0).  WC_EINVAL for
 * negative sizes, NULL arrays, or a graph in which some vertex was never
 * colored (not symmetric; such vertices keep -1); the colors of other
 * asymmetric graphs are unspecified. */
wc_status wc_color(wc_ctx *ctx, const wc_csr *g, const uint32_t *prio, int32_t *color, wc_mode mode,
                   const wc_tune *tune, hipStream_t stream, wc_stats *stats);

/* Tree descendants (recursion of Fig. 1(c)): desc[v] = number of proper
 * descendants of v.  A node with children is a recursive call whose work is
 * consolidated per `mode`; a leaf gets 0; the post-work folds each child c
 * into its parent as 1 + desc[c].
 *   WC_FLAT, WC_GRID: level-synchronous (one launch per level, a graph of all
 *     levels replayed by a repeated call), the folds by one bottom-up pass per level.
 *   WC_WAVE, WC_BLOCK: no grid-wide barrier: a persistent grid whose groups
 *     flush the calls they find as packets of about 64 * items_per_lane (wave)
 *     or block_threads * items_per_lane (block) children into a device-wide
 *     queue; a node's post-work runs when its last child finishes.  Waits for
 *     packets are bounded (WC_ETIMEOUT). */
wc_status wc_tree_descendants(wc_ctx *ctx, const wc_tree *t, int32_t *desc, wc_mode mode, const wc_tune *tune,
                              hipStream_t stream, wc_stats *stats);

/* Tree heights: height[v] = edges on the longest downward path from v (leaf 0);
 * same traversal as wc_tree_descendants with the fold max(1 + height[c]). */
wc_status wc_tree_height(wc_ctx *ctx, const wc_tree *t, int32_t *height, wc_mode mode, const wc_tune *tune,
                         hipStream_t stream, wc_stats *stats);

/* Batched tree descendants / heights: `count` trees of any sizes in one
 * sequence of level launches (a systems pattern around the method; each tree is
 * the problem of wc_tree_descendants / wc_tree_height).  trees and desc /
 * height are HOST arrays of `count` entries whose pointers are device arrays
 * (desc[i] has trees[i].n entries and is written entirely; trees[i].parent is
 * not read).  Flat or grid mode for the whole batch: every level kernel takes
 * the items of that depth in all trees, so grid mode consolidates the recursive
 * calls of all trees into one buffer per level (one child per level for the
 * whole batch) and its post-work likewise.  A call repeated with the same
 * trees, outputs, mode and tune replays a HIP graph of all its levels.
 * Results equal the single-tree calls.  WC_EINVAL for wave or block mode, a
 * tree without root, NULL arrays, more than 2^31 nodes in total, or
 * tune->driver != 0. */
wc_status wc_tree_descendants_batch(wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *desc,
                                    wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats);
wc_status wc_tree_height_batch(wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *height,
                               wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats);

/* Batched SSSP: `count` independent instances in one launch sequence
 * (a systems pattern around the method; each instance is the problem of wc_sssp).
 * graphs, w, src, dist are HOST arrays of `count` entries whose pointers are
 * device arrays of each instance (dist[i] has graphs[i].n entries and is written
 * entirely).  modes/tunes (nullable: grid mode, defaults) give each instance
 * its own consolidation granularity, threshold and items_per_lane, as chosen
 * per size bucket by an autotuner; block_threads must be equal across
 * instances.  The instances share one grid: every round, one parent kernel
 * scans all instances' vertices and each heavy vertex goes to its instance's
 * wave, block or global buffer; the global buffer consolidates the heavy work
 * of all grid-mode instances into one child.
 * graph_rounds > 0: that many rounds are captured once into a HIP graph (its
 * kernels return at once after convergence) and replayed as one graph launch
 * on later calls with the same shape; rounds beyond it run as ordinary
 * launches.  graph_rounds = 0: ordinary launches only.  Results are identical
 * to wc_sssp on each instance.  The call returns after the device has
 * published whether the rounds converged. */
wc_status wc_sssp_batch(wc_ctx *ctx, int32_t count, const wc_csr *graphs, const uint32_t *const *w,
                        const int32_t *src, uint32_t *const *dist, const wc_mode *modes, const wc_tune *tunes,
                        int32_t graph_rounds, hipStream_t stream, wc_stats *stats);

/* Size of the fixed device array that wc_spmv_noalloc uses as its workspace. */
#define WC_SPMV_NOALLOC_SCRATCH_BYTES (64u << 20)

/* wc_spmv for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product, kernels and summation order as wc_spmv with the same mode and tune
 * (so bit-identical results), but no context, no pool and no stats.  The
 * grid-mode workspace lives in one fixed device array of
 * WC_SPMV_NOALLOC_SCRATCH_BYTES per device, held from the first call on that
 * device until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.  Grid mode needs about 52 n + 20 m / (64 * items_per_lane)
 * + 72 ceil(n / block_threads) bytes (n up to about 1.2 million at m = 16 n
 * with the defaults); a call whose workspace could exceed the array returns
 * WC_EINVAL before anything is enqueued, as do bad arguments and
 * tune->driver != 0.  Flat mode uses no workspace; wave and block modes only
 * for the rows they hand on to the grid (about 0.44 m bytes with the defaults).
 * Runs on the calling thread's current device (hipSetDevice); `stream` must
 * belong to it.  The call only enqueues; the caller synchronizes.  Every call
 * on one device shares its array: calls whose stream work overlaps on one
 * device (different streams or host threads without ordering between them)
 * race and give undefined results; calls on one stream are ordered and safe.
 * Nothing in the array needs to start at zero (every piece is written before
 * it is read within a call). */
wc_status wc_spmv_noalloc(const wc_csr *a, const float *val, const float *x, float *y, wc_mode mode,
                          const wc_tune *tune, hipStream_t stream);

/* Per-kernel timing.  When enabled, a HIP event is recorded on the launch
 * stream after every kernel the library launches on a context, and before the
 * first kernel of a call (and after any other stream work of the library), so
 * each kernel's device time, dispatch gap included, can be read back
 * afterwards.  Enabling or disabling waits for the device and discards earlier
 * records. */
wc_status wc_ctx_set_timing(wc_ctx *ctx, int enable);

/* Bound of every device-side wait of later calls on this context (the packet
 * queues of the trees' wave and block modes), in microseconds; <= 0 restores
 * the default of 2 s.  A wait that passes its bound gives up and the call
 * returns WC_ETIMEOUT (its outputs are then incomplete); every kernel still
 * exits normally.  Meant for tests of the timeout path and for callers that
 * want a tighter bound.  WC_EINVAL for a NULL context. */
wc_status wc_ctx_set_wait_limit(wc_ctx *ctx, int64_t microseconds);

/* Plan-only mode, for callers that budget device memory before running (a
 * serving loop admitting work by free memory): while enabled, every call on
 * this context checks its arguments, records the pool bytes it would carve
 * (its workspace: consolidation buffers, frontier and level arrays) and
 * returns WC_PLANNED without enqueueing anything or touching the pool.
 * Enabling or disabling resets the recorded maximum.  Calls that return
 * WC_OK at once (empty inputs) need no workspace. */
wc_status wc_ctx_set_plan_only(wc_ctx *ctx, int enable);

/* Largest workspace (bytes) recorded by calls made in plan-only mode since it
 * was last switched. */
wc_status wc_ctx_planned_bytes(wc_ctx *ctx, size_t *bytes);

/* Current pool size in bytes and the number of times the pool has grown (a
 * call that needs more than the pool replaces it by one of at least twice the
 * size without waiting: calls still in flight keep the old pool, which stays
 * allocated, with the context's captured graphs, until the context next drains
 * the device: wc_ctx_set_timing or wc_ctx_destroy). */
wc_status wc_ctx_pool_info(wc_ctx *ctx, size_t *pool_bytes, int64_t *grows);

/* Grows the pool to at least `bytes` now, so that later calls up to that size
 * never grow it.  Does not wait for the device: the replaced pool and the
 * context's captured graphs are retired as a growth inside a call retires them
 * (see wc_ctx_pool_info), so until the context next drains the device both
 * pools count against device memory.  No-op when the pool is large enough. */
wc_status wc_ctx_reserve(wc_ctx *ctx, size_t bytes);

/* Aggregate of the recorded launches of the index-th distinct kernel name (in
 * first-launch order): its name (a static string), launch count, total and
 * largest event-measured duration in milliseconds.  Waits for the recorded
 * events.  Returns WC_EINVAL when index is past the last name. */
wc_status wc_ctx_kernel_stats(wc_ctx *ctx, int32_t index, const char **name, int64_t *launches, double *total_ms,
                              double *max_ms);

/* The index-th recorded launch in launch order: kernel name (static string) and
 * its event-measured duration in milliseconds.  Waits for its events.  Returns
 * WC_EINVAL past the last record. */
wc_status wc_ctx_kernel_record(wc_ctx *ctx, int32_t index, const char **name, double *ms);

/* Thread-local description of the last non-WC_OK status on this thread. */
const char *wc_last_error(void);

/* Library version string. */
const char *wc_version(void);

/* ---- host-side planning helpers (no device work; usable without a GPU) ---- */

/* Per-buffer capacity estimate of Sec. IV.E: total_thread * total_buff_var * items_per_thread. */
int64_t wc_per_buffer_size(int64_t total_thread, int64_t total_buff_var, int64_t items_per_thread);

/* KC_X of Sec. IV.E: (blocks, threads) downgraded to (ceil(blocks / x), threads). */
void wc_kc_config(int64_t blocks, int64_t threads, int64_t x, int64_t *out_blocks, int64_t *out_threads);

/* Fill `out` with the library's defaults for a problem ("sssp", "bfs", "spmv", "tree", "color")
 * and mode, given the occupancy-derived resident workgroup count ("tree" gives
 * the heights' workgroup size; the descendants at block level use 512).
 * Returns WC_EINVAL for an unknown problem or mode. */
wc_status wc_default_tune(const char *problem, wc_mode mode, int32_t resident_blocks, wc_tune *out);

#ifdef __cplusplus
}
#endif

#endif /* WC_H */
