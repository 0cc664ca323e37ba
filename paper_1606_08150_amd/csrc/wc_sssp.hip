// SSSP with workload consolidation (irregular loop of Fig. 1(b)).
//
// Frontier-driven rounds: round r expands every vertex whose distance improved
// in round r-1.  A frontier vertex is one parent work item; its prework reads
// its CSR range and current distance, and the condition of Fig. 1(b) compares
// its out-degree with the threshold.  A light vertex relaxes its edges inline
// ("work"); a heavy one is inserted into the consolidation buffer of its mode
// and relaxed by the consolidated child ("process_neighbors"):
//   wave  - the wave's ballot mask is the buffer; the whole wave then relaxes
//           the concatenated edge ranges of its buffered vertices, 64 lanes
//           side by side (no barrier).
//   block - thread-ordered LDS buffer; after the workgroup barrier the block
//           relaxes the concatenated edge ranges of all buffered vertices, each
//           thread taking every BLOCK-th edge (a multi-thread child wrapped in a
//           loop over the buffer, Sec. IV.C, load-balanced over items).
//   grid  - global buffer of (vertex, edge range) chunks of 64 * items_per_lane
//           edges, reserved with one atomic per workgroup window; after the
//           grid-wide barrier (the kernel boundary) a moldable grid drains all
//           chunks, two per wave at a time.
//   flat  - every vertex relaxes all of its edges itself.
// Relaxation: nd = dist[u] + w; atomicMin on dist[v].  Flat, wave and block
// modes put an improved vertex into the next frontier with a per-vertex round
// stamp; grid mode keeps relaxed_at[v], the distance v's edges were last
// relaxed with, and its frontier is every vertex whose distance is below it.
// The distances reached are the unique shortest-path distances, so every mode
// and schedule yields identical results.
#include <cstring>
#include <algorithm>
#include <vector>


#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

constexpr int kPad = 32;  // ring entries live on separate 128-byte lines
constexpr int kUnroll = 4;  // edges in flight per lane

struct SsspArgs {
    const int *row_ptr;
    const int *col;
    const uint32_t *w;  // nullptr: unit weights (breadth-first levels)
    uint32_t *dist;
    int *stamp;       // stamp[v] == r: v is a frontier vertex of round r
    uint32_t *relaxed_at;  // grid mode: the largest distance v's edges were last relaxed with;
                           // v is in the frontier while dist[v] is below it
    int *active;      // ring of 3 flags (stride kPad): round r has a frontier
    int *chunk_tail;  // ring of 3 grid-buffer tails (stride kPad)
    int4 *chunks;     // grid consolidation buffer: (u, begin, end, 0)
    long long chunk_cap;
    int n;
    int threshold;
    int chunk;
    int spill;        // wave and block modes: buffered items with more edges go to the global buffer
    int buffer_alloc; // wave and block buffers: 0 registers / LDS, 1 pool slices, 2 device malloc
    int4 *group_bufs; // buffer_alloc 1: one slice of BLOCK + 1 items per workgroup (waves: 64 each)
    unsigned long long *host_ring;
    DevStats *stats;
    int want_stats;
};

// Edge weight; without weights (breadth-first levels) every edge weighs 1.
__device__ __forceinline__ uint32_t weight(const SsspArgs &a, int e) { return a.w ? a.w[e] : 1u; }

__device__ __forceinline__ uint32_t add_sat(uint32_t du, uint32_t w)
{
    uint32_t s = du + w;
    return s < du ? kInf : s;
}

// Relaxes edge e of a vertex at distance du: atomicMin on dist[v]; with STAMP
// (flat, wave and block modes), v is stamped into the next round's frontier.
// dv is a plain read of dist[v] taken earlier in the round; a stale read is
// only ever too high.  The atomic's old value is not waited for: when nd < dv
// but another relaxation of this round got dist[v] below nd first, that
// relaxation stamps v too, so stamping on nd < dv gives the same frontier (and
// a vertex stamped twice is expanded once).  Grid mode keeps no stamps: its
// frontier is the set of vertices whose distance is below relaxed_at.
template <bool STAMP>
__device__ __forceinline__ bool relax_loaded(const SsspArgs &a, int v, uint32_t nd, uint32_t dv, int next)
{
    if (nd >= dv) return false;
    atomic_min_dev_noret(&a.dist[v], nd);
    if (STAMP) a.stamp[v] = next;
    return true;
}

// U edges per lane at once: e_k = first + k * stride (valid while < end).
// Loads are issued for all k before any relaxation, for memory-level parallelism.
template <bool STAMP, int U = kUnroll>
__device__ __forceinline__ int relax_batch(const SsspArgs &a, int first, int stride, int end, uint32_t du,
                                           int next)
{
    int v[U];
    uint32_t wt[U], dv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int e = first + k * stride;
        const bool ok = e < end;
        v[k] = ok ? a.col[e] : -1;
        wt[k] = ok ? weight(a, e) : 0u;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) dv[k] = v[k] >= 0 ? a.dist[v[k]] : 0u;
    int upd = 0;
#pragma unroll
    for (int k = 0; k < U; ++k)
        if (v[k] >= 0) upd += relax_loaded<STAMP>(a, v[k], add_sat(du, wt[k]), dv[k], next);
    return upd;
}

// Inline "work" of Fig. 1(b): the lane relaxes edges [beg, end) of its vertex,
// 2 * kUnroll at a time (a light vertex of the default threshold in one step).
template <bool STAMP>
__device__ __forceinline__ int relax_lane(const SsspArgs &a, int beg, int end, uint32_t du, int next)
{
    int upd = 0;
    for (int e = beg; e < end; e += 2 * kUnroll) upd += relax_batch<STAMP, 2 * kUnroll>(a, e, 1, end, du, next);
    return upd;
}

// Two chunks of the grid buffer at once (uniform arguments): each lane keeps
// 2 * kUnroll edges in flight.  The chunks' source distances are read after
// their edges are requested (they may have improved since the vertex was
// buffered); the largest distance used per chunk is returned.  Chunk 1 may be
// empty (cb1 == ce1, u1 unused).
template <bool STAMP>
__device__ __forceinline__ int relax_wave2(const SsspArgs &a, int u0, int cb0, int ce0, int u1, int cb1, int ce1,
                                            int next, uint32_t &du0_used, uint32_t &du1_used)
{
    int upd = 0;
    const int len = max(ce0 - cb0, ce1 - cb1);
    du0_used = 0u;
    du1_used = 0u;
    for (int o = lane_id(); o - lane_id() < len; o += kWave * kUnroll) {
        int v[2 * kUnroll];
        uint32_t wt[2 * kUnroll], dv[2 * kUnroll];
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k) {
            const int e = (k < kUnroll ? cb0 : cb1) + o + (k % kUnroll) * kWave;
            const bool ok = e < (k < kUnroll ? ce0 : ce1);
            v[k] = ok ? a.col[e] : -1;
            wt[k] = ok ? weight(a, e) : 0u;
        }
        const uint32_t du0 = a.dist[u0];
        const uint32_t du1 = cb1 < ce1 ? a.dist[u1] : 0u;
        du0_used = max(du0_used, du0);
        du1_used = max(du1_used, du1);
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k) dv[k] = v[k] >= 0 ? a.dist[v[k]] : 0u;
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k)
            if (v[k] >= 0) upd += relax_loaded<STAMP>(a, v[k], add_sat(k < kUnroll ? du0 : du1, wt[k]), dv[k], next);
    }
    return upd;
}

__device__ __forceinline__ void mark_active(const SsspArgs &a, int r, bool any)
{
    if (__ballot(any) && lane_id() == 0) a.active[((r + 1) % 3) * kPad] = 1;
}

// Child thread-count heuristic of the wave and block modes (the KC_X rule of
// Sec. IV.E: a warp's or block's consolidated child is launched with many
// blocks, not just the parent group's threads).  An item of the wave's or
// block's buffer with more than `spill` edges (one chunk) is handed on as
// chunks of the round's global buffer, which the drain kernel after the
// parent spreads over the whole grid, instead of occupying its own group for
// its whole edge list.
// Every lane of the wave calls this (nch = 0: nothing to hand on); one atomic
// per wave reserves the slots and the wave writes each item's chunks together.
// A chunk beyond the buffer's capacity is relaxed by the writing lane itself
// (the overflow fallback).  Returns the updates made by such fallbacks.
__device__ __forceinline__ int spill_chunks(const SsspArgs &a, int r, int u, int beg, int end, uint32_t du, int nch)
{
    const int slot = wave_reserve_n(nch, &a.chunk_tail[(r % 3) * kPad]);
    int upd = 0;
    uint64_t m = __ballot(nch > 0);
    while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int s0 = readlane(slot, b), n0 = readlane(nch, b), rb = readlane(beg, b), re = readlane(end, b);
        const int ub = readlane(u, b);
        const uint32_t dub = readlane_u(du, b);
        for (int c = lane_id(); c < n0; c += kWave) {
            const int cb = rb + c * a.chunk, ce = min(re, cb + a.chunk);
            if ((long long)s0 + c < a.chunk_cap) {
                a.chunks[s0 + c] = make_int4(ub, cb, ce, 0);
            } else {
                a.stats->overflowed = 1;
                upd += relax_lane<true>(a, cb, ce, dub, r + 1);
            }
        }
    }
    return upd;
}

// The consolidated child of a wave (G = 64) or a block (G = BLOCK) over its
// buffer of nb items: item i holds edges [beg_i, beg_i + deg_i) of a vertex at
// distance du_i, and pre_i is the exclusive prefix of the degrees (total in
// all).  The group relaxes the concatenated edge ranges, G * kUnroll edges per
// step, thread t taking flattened edges t, t + G, ...: each thread finds the
// item of its edge with a cursor that only moves forward, so the lanes stay
// busy however the degrees are spread over the items.
template <int G>
__device__ __forceinline__ int relax_items(const SsspArgs &a, const int *ibeg, const uint32_t *idu, const int *ipre,
                                           int nb, int total, int t, int next)
{
    int upd = 0, it = 0;
    for (int j0 = t; j0 < total; j0 += G * kUnroll) {
        int v[kUnroll];
        uint32_t nd[kUnroll], dv[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            const int j = j0 + q * G;
            v[q] = -1;
            nd[q] = 0;
            if (j < total) {
                while (it + 1 < nb && ipre[it + 1] <= j) ++it;
                const int e = ibeg[it] + (j - ipre[it]);
                v[q] = a.col[e];
                nd[q] = add_sat(idu[it], weight(a, e));
            }
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) dv[q] = v[q] >= 0 ? a.dist[v[q]] : 0u;
#pragma unroll
        for (int q = 0; q < kUnroll; ++q)
            if (v[q] >= 0) upd += relax_loaded<true>(a, v[q], nd[q], dv[q], next);
    }
    return upd;
}

// relax_items over a buffer in global memory: item i is (beg, du, pre, 0).
template <int G>
__device__ __forceinline__ int relax_items_global(const SsspArgs &a, const int4 *gb, int nb, int total, int t,
                                                  int next)
{
    int upd = 0, it = 0;
    for (int j0 = t; j0 < total; j0 += G * kUnroll) {
        int v[kUnroll];
        uint32_t nd[kUnroll], dv[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            const int j = j0 + q * G;
            v[q] = -1;
            nd[q] = 0;
            if (j < total) {
                while (it + 1 < nb && gb[it + 1].z <= j) ++it;
                const int4 d = gb[it];
                const int e = d.x + (j - d.z);
                v[q] = a.col[e];
                nd[q] = add_sat((uint32_t)d.y, weight(a, e));
            }
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) dv[q] = v[q] >= 0 ? a.dist[v[q]] : 0u;
#pragma unroll
        for (int q = 0; q < kUnroll; ++q)
            if (v[q] >= 0) upd += relax_loaded<true>(a, v[q], nd[q], dv[q], next);
    }
    return upd;
}

// Buffers in global memory, for the allocator comparison of Sec. V.A: the
// paper's consolidation buffers live in global memory and come either from a
// pre-allocated pool or from the device's malloc.  Here the group writes its
// buffered items out, its child reads them back, and a malloc'ed buffer is
// freed after the child.  A failed malloc leaves the items in registers / LDS
// (the default path) and raises the overflow flag.
__device__ __forceinline__ int4 *group_buffer(const SsspArgs &a, int slot, int items)
{
    if (a.buffer_alloc == 1) return a.group_bufs + slot;
    return static_cast<int4 *>(malloc((size_t)items * sizeof(int4)));
}

// Wave mode: the items of the lanes in `mask` (pre: exclusive prefix of their
// degrees, total in all) through a global buffer.
__device__ __forceinline__ int wave_child_global(const SsspArgs &a, uint64_t mask, bool mine, int beg, int pre,
                                                 int total, uint32_t du, int next, bool &done)
{
    const int nb = __builtin_popcountll(mask);
    unsigned long long p = 0;
    if (lane_id() == 0) {
        // pool slices: the block's slice of BLOCK + 1 items, 64 per wave
        const int wave_slot = blockIdx.x * (blockDim.x + 1) + threadIdx.x / kWave * kWave;
        p = reinterpret_cast<unsigned long long>(group_buffer(a, wave_slot, nb));
    }
    p = ((unsigned long long)readlane_u((uint32_t)(p >> 32), 0) << 32) | readlane_u((uint32_t)p, 0);
    int4 *buf = reinterpret_cast<int4 *>(p);
    done = buf != nullptr;
    if (!buf) {
        if (lane_id() == 0) a.stats->overflowed = 1;
        return 0;
    }
    if (mine) buf[rank_in(mask)] = make_int4(beg, (int)du, pre, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int upd = relax_items_global<kWave>(a, buf, nb, total, lane_id(), next);
    if (a.buffer_alloc == 2 && lane_id() == 0) free(buf);
    return upd;
}

// A wave's buffer in LDS (wave mode): up to 64 items per wave.
template <int BLOCK>
struct WaveBuf {
    int beg[BLOCK / kWave][kWave];
    uint32_t du[BLOCK / kWave][kWave];
    int pre[BLOCK / kWave][kWave];
};

template <int BLOCK>
struct BlockBuf {
    int beg[BLOCK];
    uint32_t du[BLOCK];
    int pre[BLOCK + 1];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
    int4 *gbuf;  // buffer_alloc != 0: the block's buffer in global memory (or NULL: LDS)
};

// Parent kernel of round r in flat, wave and block modes: thread i takes vertex
// i (Fig. 1(b)); the vertices stamped r form the frontier.  Grid-stride windows
// of BLOCK vertices; every thread of a block runs the same number of windows.
// ALLOC: the instantiation with the global-memory buffers of the allocator
// comparison (pool slices or device malloc); the device-malloc call needs so
// many registers that it is kept out of the default kernels (which then run
// 7 waves per SIMD instead of 4).
template <int MODE, int BLOCK, bool ALLOC = false>
__global__ __launch_bounds__(BLOCK) void sssp_round(SsspArgs a, int r)
{
    const int act = a.active[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.active[((r + 2) % 3) * kPad] = 0;
        a.chunk_tail[((r + 1) % 3) * kPad] = 0;
        publish_host(a.host_ring, r % kHostRing, a.stats, act);
    }
    if (!act) return;
    const int next = r + 1;
    const int lane = lane_id();
    StatAcc acc;
    for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {
        const int u = base + threadIdx.x;
        const bool member = u < a.n && a.stamp[u] == r;
        int beg = 0, end = 0;
        uint32_t du = 0;
        if (member) {
            beg = a.row_ptr[u];
            end = a.row_ptr[u + 1];
            du = a.dist[u];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        if (a.want_stats) {
            acc.edges += deg;
            acc.buffered += heavy ? deg : 0;
            acc.items += heavy ? 1 : 0;
            if (MODE == WC_WAVE && __ballot(heavy) && lane == 0) acc.dispatches += 1;
        }
        // work: light items relax inline
        const int upd_inline = relax_lane<true>(a, beg, heavy ? beg : end, du, next);
        int upd = 0;  // by the consolidated child

        // buffered items too long for the group's own child go to the global buffer
        const bool spill = MODE != WC_FLAT && heavy && deg > a.spill;
        if constexpr (MODE != WC_FLAT) {
            if (__ballot(spill)) upd += spill_chunks(a, r, u, beg, end, du, spill ? (deg + a.chunk - 1) / a.chunk : 0);
        }
        const bool mine = heavy && !spill;

        if constexpr (MODE == WC_WAVE) {
            // insert_buffer = ballot: the mask is the wave's buffer and the lanes'
            // ranks order it; no barrier is needed within one wave
            const uint64_t mask = __ballot(mine);
            if (mask) {
                const int incl = wave_incl_scan(mine ? deg : 0);
                const int total = readlane(incl, kWave - 1), pre = incl - (mine ? deg : 0);
                bool done = false;
                if constexpr (ALLOC) upd += wave_child_global(a, mask, mine, beg, pre, total, du, next, done);
                if (!done) {
                    __shared__ WaveBuf<BLOCK> wb;
                    const int w = threadIdx.x / kWave;
                    if (mine) {
                        const int k = rank_in(mask);
                        wb.beg[w][k] = beg;
                        wb.du[w][k] = du;
                        wb.pre[w][k] = pre;
                    }
                    wave_lds_sync();
                    upd += relax_items<kWave>(a, wb.beg[w], wb.du[w], wb.pre[w], __builtin_popcountll(mask), total,
                                              lane, next);
                    wave_lds_sync();  // the next window rewrites the wave's entries
                }
            }
        } else if constexpr (MODE == WC_BLOCK) {
            __shared__ BlockBuf<BLOCK> sb;
            int k, off, nb, total;
            block_scan2<BLOCK>(mine ? 1 : 0, mine ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if constexpr (ALLOC) {
                // the buffer in global memory (allocator comparison); NULL: LDS
                if (threadIdx.x == 0) {
                    sb.gbuf = nb ? group_buffer(a, blockIdx.x * (BLOCK + 1), nb + 1) : nullptr;
                    if (nb && !sb.gbuf) a.stats->overflowed = 1;
                }
                __syncthreads();
            }
            int4 *const gb = ALLOC ? sb.gbuf : nullptr;
            if (mine) {
                if (gb) {
                    gb[k] = make_int4(beg, (int)du, off, 0);
                } else {
                    sb.beg[k] = beg;
                    sb.du[k] = du;
                    sb.pre[k] = off;
                }
            }
            if (threadIdx.x == 0) {
                if (gb) gb[nb] = make_int4(0, 0, total, 0);
                else sb.pre[nb] = total;
            }
            // the block's buffer counts as one dispatch when it holds any item,
            // also when all of them were handed on to the grid
            if (a.want_stats && __syncthreads_or(heavy) && threadIdx.x == 0) acc.dispatches += 1;
            __syncthreads();  // the "synchronize" between inserts and the child
            // the block relaxes the concatenated edge ranges of its items
            if (ALLOC && gb) upd += relax_items_global<BLOCK>(a, gb, nb, total, threadIdx.x, next);
            else upd += relax_items<BLOCK>(a, sb.beg, sb.du, sb.pre, nb, total, threadIdx.x, next);
            __syncthreads();  // LDS buffer is reused by the next window
            if constexpr (ALLOC)
                if (gb && a.buffer_alloc == 2 && threadIdx.x == 0) free(gb);
        }
        if (a.want_stats) {
            acc.updates += upd_inline + upd;
            acc.updates_buffered += upd;
        }
        mark_active(a, r, upd_inline + upd > 0);
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Two light vertices' inline work at once: each lane keeps kUnroll edges of
// each vertex in flight.
__device__ __forceinline__ int relax_lane2(const SsspArgs &a, int b0, int e0, uint32_t du0, int b1, int e1,
                                            uint32_t du1, int next)
{
    constexpr int U = kUnroll;
    int upd = 0;
    const int len = max(e0 - b0, e1 - b1);
    for (int o = 0; o < len; o += U) {
        int v[2 * U];
        uint32_t nd[2 * U], dv[2 * U];
#pragma unroll
        for (int k = 0; k < 2 * U; ++k) {
            const int e = (k < U ? b0 : b1) + o + (k % U);
            const bool ok = e < (k < U ? e0 : e1);
            v[k] = ok ? a.col[e] : -1;
            nd[k] = ok ? add_sat(k < U ? du0 : du1, weight(a, e)) : 0u;
        }
#pragma unroll
        for (int k = 0; k < 2 * U; ++k) dv[k] = v[k] >= 0 ? a.dist[v[k]] : 0u;
#pragma unroll
        for (int k = 0; k < 2 * U; ++k)
            if (v[k] >= 0) upd += relax_loaded<false>(a, v[k], nd[k], dv[k], next);
    }
    return upd;
}

// Parent kernel of grid mode.  As sssp_round, but every thread takes two
// vertices of a window of 2 * BLOCK (u and u + BLOCK), with the loads of both
// issued together: the parent is bound by the latency of its dependent loads
// (frontier test, then CSR range and distance, then edges, then targets).
// STATS: the instantiation that counts work for wc_stats; without it the
// kernel keeps no counters live and fits its registers without spilling.
template <int BLOCK, bool STATS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void sssp_round_grid2(SsspArgs a,
                                                                                         int r)
{
    constexpr int V = 2;
    __shared__ int s_tmp[2 * (BLOCK / kWave)];
    __shared__ int s_base;
    __shared__ int s_excl[V * BLOCK], s_beg[V * BLOCK], s_end[V * BLOCK];
    __shared__ uint32_t s_du[V * BLOCK];
    const int act = a.active[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.active[((r + 2) % 3) * kPad] = 0;
        a.chunk_tail[((r + 1) % 3) * kPad] = 0;
        publish_host(a.host_ring, r % kHostRing, a.stats, act);
    }
    if (!act) return;
    const int next = r + 1;
    StatAcc acc;
    // Frontier of grid mode: the vertices whose distance is below relaxed_at
    // (improved since their edges were last relaxed); no stamps are kept.  The
    // test for S windows is read together, and a block skips all S at once
    // when none of them holds a frontier vertex (late rounds scan an almost
    // empty frontier).
    constexpr int S = 4;
    const int stride = gridDim.x * V * BLOCK;
    for (long long wbase = (long long)blockIdx.x * V * BLOCK; wbase < a.n; wbase += (long long)S * stride) {
        int bits = 0;
#pragma unroll
        for (int w = 0; w < S; ++w)
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const long long uu = wbase + (long long)w * stride + k * BLOCK + threadIdx.x;
                if (uu < a.n && a.dist[uu] < a.relaxed_at[uu]) bits |= 1 << (w * V + k);
            }
        if (!__syncthreads_or(bits)) continue;
        for (int w = 0; w < S; ++w) {
            const long long base_l = wbase + (long long)w * stride;
            if (base_l >= a.n) break;  // uniform in the block
            const int base = (int)base_l;
            int u[V], beg[V], end[V], nch[V];
            uint32_t du[V];
            bool member[V], heavy[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                u[k] = base + k * BLOCK + threadIdx.x;
                member[k] = (bits >> (w * V + k)) & 1;
            }
#pragma unroll
            for (int k = 0; k < V; ++k) {
                beg[k] = end[k] = 0;
                du[k] = 0;
                if (member[k]) {
                    beg[k] = a.row_ptr[u[k]];
                    end[k] = a.row_ptr[u[k] + 1];
                    du[k] = a.dist[u[k]];  // read again: it may have improved since the test
                }
            }
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const int deg = end[k] - beg[k];
                heavy[k] = deg > a.threshold;
                nch[k] = heavy[k] ? (deg + a.chunk - 1) / a.chunk : 0;
                if (STATS) {
                    acc.edges += deg;
                    acc.buffered += heavy[k] ? deg : 0;
                    acc.items += heavy[k] ? 1 : 0;
                }
            }
            // work: light items relax inline
            const int upd_inline = relax_lane2(a, beg[0], heavy[0] ? beg[0] : end[0], du[0], beg[1],
                                               heavy[1] ? beg[1] : end[1], du[1], next);
            if (STATS) acc.updates += upd_inline;
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (end[k] > beg[k] && !heavy[k]) a.relaxed_at[u[k]] = du[k];
            // most windows of a small frontier hold no heavy vertex: skip the scan
            if (!__syncthreads_or((heavy[0] || heavy[1]) ? 1 : 0)) {
                mark_active(a, r, upd_inline > 0);
                continue;
            }
            int upd_over = 0;  // chunks that did not fit, relaxed here
            int excl, d0, tot, d1;
            block_scan2<BLOCK>(nch[0] + nch[1], 0, s_tmp, excl, d0, tot, d1);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const int q = threadIdx.x * V + k;  // entries in (thread, vertex) order
                s_excl[q] = excl + (k == 0 ? 0 : nch[0]);
                s_beg[q] = beg[k];
                s_end[q] = end[k];
                s_du[q] = du[k];
            }
            if (threadIdx.x == 0) s_base = tot ? atomic_add_dev(&a.chunk_tail[(r % 3) * kPad], tot) : 0;
            __syncthreads();
            const int slot0 = s_base;
            // a heavy vertex's chunks raise relaxed_at to the distances they use
            // (drain atomics, next kernel); a chunk that overflows is relaxed here
            // with the parent's reading
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (heavy[k]) {
                    const long long last = (long long)slot0 + s_excl[threadIdx.x * V + k] + nch[k];
                    a.relaxed_at[u[k]] = last > a.chunk_cap ? du[k] : 0u;
                }
            // the block writes the window's chunks together: chunk j belongs to the
            // last entry whose offset is <= j
            for (int j = threadIdx.x; j < tot; j += BLOCK) {
                int lo = 0, hi = V * BLOCK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_excl[mid] <= j) lo = mid;
                    else hi = mid - 1;
                }
                const int cb = s_beg[lo] + (j - s_excl[lo]) * a.chunk;
                const int ce = min(s_end[lo], cb + a.chunk);
                if ((long long)slot0 + j < a.chunk_cap) {
                    a.chunks[slot0 + j] = make_int4(base + (lo % V) * BLOCK + lo / V, cb, ce, 0);
                } else {
                    // buffer full: this chunk is processed inline (fallback)
                    a.stats->overflowed = 1;
                    upd_over += relax_lane<false>(a, cb, ce, s_du[lo], next);
                }
            }
            __syncthreads();  // the LDS arrays are rewritten by the next window
            if (STATS) {
                acc.updates += upd_over;
                acc.updates_buffered += upd_over;
            }
            mark_active(a, r, upd_inline + upd_over > 0);
        }
    }
    if (STATS) stat_flush(a.stats, acc);
}

// Consolidated child of grid-level consolidation: one wave per chunk, chunks
// fetched grid-stride until the buffer is exhausted (moldable).  With STAMP
// (wave and block modes) it drains the items their groups handed on, and
// stamps improved vertices into the next frontier instead of keeping
// relaxed_at.
template <int BLOCK, bool STAMP>
__global__ __launch_bounds__(BLOCK) void sssp_drain(SsspArgs a, int r)
{
    if (!a.active[(r % 3) * kPad]) return;
    const int tail = a.chunk_tail[(r % 3) * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    const int next = r + 1;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    // in wave and block modes the drain runs the children of the groups' buffers,
    // which those groups already counted as dispatches
    if (!STAMP && a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0)
        atomic_add_dev(&a.stats->rep[0].dispatches, 1ull);
    int upd = 0;
    // two chunks per wave and step; the next pair's entries are fetched before
    // the current pair's edges
    int4 d0 = load_or_zero(a.chunks, gw, gw < total);
    int4 d1 = load_or_zero(a.chunks, gw + nw, gw + nw < total);
    for (int c = gw; c < total; c += 2 * nw) {
        const int u0 = __builtin_amdgcn_readfirstlane(d0.x), u1 = __builtin_amdgcn_readfirstlane(d1.x);
        const int cb0 = __builtin_amdgcn_readfirstlane(d0.y), ce0 = __builtin_amdgcn_readfirstlane(d0.z);
        const int cb1 = __builtin_amdgcn_readfirstlane(d1.y), ce1 = __builtin_amdgcn_readfirstlane(d1.z);
        const int cn = c + 2 * nw;
        d0 = load_or_zero(a.chunks, cn, cn < total);
        d1 = load_or_zero(a.chunks, cn + nw, cn + nw < total);
        uint32_t du0, du1;
        upd += relax_wave2<STAMP>(a, u0, cb0, ce0, u1, cb1, ce1, next, du0, du1);
        if (!STAMP && lane_id() == 0) {
            atomic_max_dev_noret(&a.relaxed_at[u0], du0);
            if (cb1 < ce1) atomic_max_dev_noret(&a.relaxed_at[u1], du1);
        }
    }
    mark_active(a, r, upd > 0);
    if (a.want_stats) {
        StatAcc acc;
        acc.updates = acc.updates_buffered = (unsigned int)upd;
        stat_flush(a.stats, acc);
    }
}

// basic dynamic parallelism, emulated for comparison (driver 2): the child of
// ONE buffered vertex, thread-mapped over its edges, launched per vertex by
// the host.  Same relaxation as the drain.
__global__ __launch_bounds__(256) void sssp_child_basic(SsspArgs a, int r, int u, int beg, int end)
{
    const int e = beg + blockIdx.x * 256 + threadIdx.x;
    const uint32_t du = a.dist[u];
    int upd = 0;
    if (e < end) {
        const int v = a.col[e];
        upd = relax_loaded<false>(a, v, add_sat(du, weight(a, e)), a.dist[v], r + 1);
    }
    if (threadIdx.x == 0) atomic_max_dev_noret(&a.relaxed_at[u], du);
    mark_active(a, r, upd > 0);
}

__global__ void sssp_init(SsspArgs a, int src)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < a.n; i += gridDim.x * blockDim.x) {
        a.dist[i] = i == src ? 0u : kInf;
        if (a.stamp) a.stamp[i] = i == src ? 0 : -1;
        if (a.relaxed_at) a.relaxed_at[i] = kInf;
    }
    if (blockIdx.x == 0 && threadIdx.x < 3) {
        a.active[threadIdx.x * kPad] = threadIdx.x == 0 ? 1 : 0;
        a.chunk_tail[threadIdx.x * kPad] = 0;
    }
}

// ---- host side --------------------------------------------------------------------------------

struct KernelSet {
    const void *round, *drain;
};

template <int BLOCK>
KernelSet pick_block(wc_mode mode, bool alloc, bool stats)
{
    const void *drain = reinterpret_cast<const void *>(&sssp_drain<BLOCK, false>);
    const void *drain_stamp = reinterpret_cast<const void *>(&sssp_drain<BLOCK, true>);
    switch (mode) {
    case WC_FLAT: return {reinterpret_cast<const void *>(&sssp_round<WC_FLAT, BLOCK>), nullptr};
    case WC_WAVE:
        return {alloc ? reinterpret_cast<const void *>(&sssp_round<WC_WAVE, BLOCK, true>)
                      : reinterpret_cast<const void *>(&sssp_round<WC_WAVE, BLOCK>),
                drain_stamp};
    case WC_BLOCK:
        return {alloc ? reinterpret_cast<const void *>(&sssp_round<WC_BLOCK, BLOCK, true>)
                      : reinterpret_cast<const void *>(&sssp_round<WC_BLOCK, BLOCK>),
                drain_stamp};
    default:
        return {stats ? reinterpret_cast<const void *>(&sssp_round_grid2<BLOCK, true>)
                      : reinterpret_cast<const void *>(&sssp_round_grid2<BLOCK, false>),
                drain};
    }
}

const char *round_name(wc_mode mode)
{
    static const char *names[] = {"sssp_round_flat", "sssp_round_wave", "sssp_round_block", "sssp_round_grid"};
    return names[mode];
}

KernelSet pick(wc_mode mode, int block, bool alloc = false, bool stats = false)
{
    switch (block) {
    case 64: return pick_block<64>(mode, alloc, stats);
    case 128: return pick_block<128>(mode, alloc, stats);
    case 512: return pick_block<512>(mode, alloc, stats);
    case 1024: return pick_block<1024>(mode, alloc, stats);
    default: return pick_block<256>(mode, alloc, stats);
    }
}

}  // namespace
}  // namespace wc

using namespace wc;

namespace wc {
namespace {

// Shortest paths from src with weights w, or breadth-first levels when w is
// NULL (every edge weighs 1).  Arguments are validated by the callers.
wc_status run_sssp(wc_ctx *ctx, const wc_csr *g, const uint32_t *w, int32_t src, uint32_t *dist, wc_mode mode,
                   const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    WC_HIP(hipSetDevice(ctx->device));

    Config cfg;
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    KernelSet ks = pick(mode, block);
    int resident = resident_blocks(ctx, ks.round, block);
    wc_status st = resolve_tune(ctx, "sssp", mode, tune, resident, &cfg);
    if (st != WC_OK) return st;
    if ((cfg.driver == 2 || cfg.driver == 3) && mode != WC_GRID)
        return fail(WC_EINVAL, "drivers 2 and 3 are comparison variants of grid mode only");
    if (cfg.buffer_alloc != 0 && mode != WC_WAVE && mode != WC_BLOCK)
        return fail(WC_EINVAL, "buffer_alloc applies to the wave and block modes only");
    ks = pick(mode, cfg.block, cfg.buffer_alloc != 0, stats != nullptr);
    resident = resident_blocks(ctx, ks.round, cfg.block);
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    // Grid buffer: every frontier vertex (at most n per round) yields at most
    // ceil(deg / chunk) chunks, so n + m / chunk + 1 entries never overflow.
    long long cap_full = n + m / chunk + 1;
    // wave and block modes hand on only vertices above `spill` edges, each at
    // most once per round: m / chunk + m / spill + 1 entries suffice
    const int spill = chunk;
    if (mode == WC_WAVE || mode == WC_BLOCK) cap_full = m / chunk + m / spill + 1;
    long long cap = mode != WC_FLAT ? (cfg.buf_capacity > 0 ? std::min(cfg.buf_capacity, cap_full) : cap_full) : 1;
    const int grid_cap = std::max(1, std::min(cfg.grid, resident));
    const long long slices = cfg.buffer_alloc == 1 ? (long long)grid_cap * (cfg.block + 1) : 0;
    size_t need = padded(n * 4) + 2 * padded(3 * kPad * 4) + padded(cap * 16) + padded(slices * 16);
    st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    SsspArgs a;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.w = w;
    a.dist = dist;
    // the frontier: round stamps (flat, wave, block) or relaxed_at (grid)
    a.stamp = mode == WC_GRID ? nullptr : pool_take<int>(ctx, n);
    a.relaxed_at = mode == WC_GRID ? pool_take<uint32_t>(ctx, n) : nullptr;
    a.active = pool_take<int>(ctx, 3 * kPad);
    a.chunk_tail = pool_take<int>(ctx, 3 * kPad);
    a.chunks = pool_take<int4>(ctx, cap);
    a.chunk_cap = cap;
    a.buffer_alloc = cfg.buffer_alloc;
    a.group_bufs = slices ? pool_take<int4>(ctx, slices) : nullptr;
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.chunk = chunk;
    // a group's own child keeps items of up to one chunk (measured at scale 22:
    // 4 chunks for a wave and one per wave for a block took 6.0 / 6.6 ms, one
    // chunk 3.8 / 4.0 ms)
    a.spill = spill;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;

    const long long per_window = mode == WC_GRID ? 2LL * cfg.block : cfg.block;
    const int windows = (int)((n + per_window - 1) / per_window);
    // Wave and block modes launch the parent with a thread per vertex (one
    // window per workgroup, as Fig. 1(b)'s parent) unless grid_blocks caps it:
    // the hardware hands the windows to CUs as they free up, which evens out
    // the windows dense with buffered vertices (scale-22 graph: wave 2.28 ->
    // 2.12 ms, block 2.49 -> 2.19 ms against the resident grid).  The pool
    // slices of the allocator comparison are per resident workgroup, so those
    // runs keep the resident grid.
    const bool own_grid = tune && tune->grid_blocks > 0;
    int grid = std::max(1, std::min(std::min(cfg.grid, resident), windows));
    if ((mode == WC_WAVE || mode == WC_BLOCK) && cfg.buffer_alloc == 0)
        grid = std::max(1, own_grid ? std::min(cfg.grid, windows) : windows);
    const int dgrid = std::max(1, std::min(cfg.grid, resident));
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    int init_grid = (int)std::min<long long>((n + 255) / 256, 4096);
    {
        void *args[] = {&a, &src};
        st = launch(ctx, "sssp_init", reinterpret_cast<const void *>(&sssp_init), dim3(init_grid), dim3(256), args,
                    stream);
        if (st != WC_OK) return st;
    }
    if (cfg.driver == 2) {
        // Basic dynamic parallelism, emulated: after each parent round the host
        // reads the buffered vertices back and launches one child per vertex
        // (no consolidation), then waits for the round to end.
        std::vector<int4> items;
        int rounds = 0;
        for (int r = 0;; ++r) {
            void *args[] = {&a, &r};
            st = launch(ctx, "sssp_round_grid", ks.round, dim3(grid), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            int tail = 0, act = 0;
            WC_HIP(hipMemcpyAsync(&tail, a.chunk_tail + (r % 3) * kPad, sizeof(int), hipMemcpyDeviceToHost, stream));
            WC_HIP(hipStreamSynchronize(stream));
            const int count = (int)std::min<long long>(tail, a.chunk_cap);
            items.resize((size_t)std::max(count, 1));
            if (count > 0)
                WC_HIP(hipMemcpy(items.data(), a.chunks, sizeof(int4) * (size_t)count, hipMemcpyDeviceToHost));
            chain_break(ctx);
            long long launches = 0;
            for (int i = 0; i < count;) {
                // a vertex's chunks are consecutive: one child over all its edges
                int j = i + 1;
                while (j < count && items[j].x == items[i].x && items[j].y == items[j - 1].z) ++j;
                int u = items[i].x, beg = items[i].y, end = items[j - 1].z;
                void *cargs[] = {&a, &r, &u, &beg, &end};
                st = launch(ctx, "sssp_child_basic", reinterpret_cast<const void *>(&sssp_child_basic),
                            dim3((end - beg + 255) / 256), dim3(256), cargs, stream);
                if (st != WC_OK) return st;
                ++launches;
                i = j;
            }
            if (stats) stats->dispatches += launches;
            WC_HIP(hipMemcpyAsync(&act, a.active + ((r + 1) % 3) * kPad, sizeof(int), hipMemcpyDeviceToHost, stream));
            WC_HIP(hipStreamSynchronize(stream));
            chain_break(ctx);
            ++rounds;
            if (!act) break;
            if (rounds > n + 1) return fail(WC_ETIMEOUT, "wc_sssp: more rounds than vertices");
        }
        const int64_t launches = stats ? stats->dispatches : 0;
        st = end_call(ctx, stream, stats, rounds, cfg.fail_on_overflow);
        if (stats) stats->dispatches = launches;
        return st;
    }
    if (cfg.driver == 3) {
        // 1-1 mapping (Sec. V.B, for comparison): the consolidated child is
        // launched with one wave per buffered chunk instead of the resident
        // grid, which needs the buffer's size on the host after every parent.
        const int waves_per_block = cfg.block / kWave;
        int rounds = 0;
        for (int r = 0;; ++r) {
            void *args[] = {&a, &r};
            st = launch(ctx, "sssp_round_grid", ks.round, dim3(grid), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            int tail = 0, act = 0;
            WC_HIP(hipMemcpyAsync(&tail, a.chunk_tail + (r % 3) * kPad, sizeof(int), hipMemcpyDeviceToHost, stream));
            WC_HIP(hipStreamSynchronize(stream));
            chain_break(ctx);
            const long long count = std::min<long long>(tail, a.chunk_cap);
            const int blocks = (int)std::max<long long>(1, (count + waves_per_block - 1) / waves_per_block);
            st = launch(ctx, "sssp_drain", ks.drain, dim3(blocks), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            WC_HIP(hipMemcpyAsync(&act, a.active + ((r + 1) % 3) * kPad, sizeof(int), hipMemcpyDeviceToHost, stream));
            WC_HIP(hipStreamSynchronize(stream));
            chain_break(ctx);
            ++rounds;
            if (!act) break;
            if (rounds > n + 1) return fail(WC_ETIMEOUT, "wc_sssp: more rounds than vertices");
        }
        return end_call(ctx, stream, stats, rounds, cfg.fail_on_overflow);
    }
    // Relaunch driver: keep `window` rounds in flight; each round kernel
    // publishes whether its frontier is non-empty to pinned host memory, and the
    // first empty round ends the loop (rounds already enqueued behind it find
    // no frontier and return at once).
    const int window = 4;
    int rounds = 0, launched = 0;
    for (;;) {
        while (launched < rounds + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, round_name(mode), ks.round, dim3(grid), dim3(cfg.block), args, stream);
            if (st == WC_OK && ks.drain)
                st = launch(ctx, "sssp_drain", ks.drain, dim3(dgrid), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            ++launched;
        }
        int c = 0;
        st = wait_round_count(ctx, rounds, &c);
        if (st != WC_OK) return st;
        if (c == 0) break;
        ++rounds;
        if (rounds > n + 1) return fail(WC_ETIMEOUT, "wc_sssp: more rounds than vertices");
    }
    return end_call(ctx, stream, stats, rounds, cfg.fail_on_overflow);
}

// Validation shared by both entry points.
wc_status check_args(const char *who, wc_ctx *ctx, const wc_csr *g, int32_t src, const uint32_t *dist, wc_mode mode)
{
    const std::string w(who);
    if (!ctx || !g) return fail(WC_EINVAL, w + ": NULL context or graph");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, w + ": bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, w + ": negative size");
    if (g->n > 0 && (src < 0 || src >= g->n)) return fail(WC_EINVAL, w + ": source out of range");
    if (g->n > 0 && (!g->row_ptr || !dist || (g->m > 0 && !g->col))) return fail(WC_EINVAL, w + ": NULL array");
    return WC_OK;
}

}  // namespace
}  // namespace wc

extern "C" wc_status wc_sssp(wc_ctx *ctx, const wc_csr *g, const uint32_t *w, int32_t src, uint32_t *dist,
                             wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    wc_status st = check_args("wc_sssp", ctx, g, src, dist, mode);
    if (st != WC_OK) return st;
    if (g->n > 0 && g->m > 0 && !w) return fail(WC_EINVAL, "wc_sssp: NULL weights");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    // without edges w may be NULL: the result does not depend on weights
    return run_sssp(ctx, g, w, src, dist, mode, tune, stream, stats);
}

extern "C" wc_status wc_bfs(wc_ctx *ctx, const wc_csr *g, int32_t src, uint32_t *level, wc_mode mode,
                            const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    wc_status st = check_args("wc_bfs", ctx, g, src, level, mode);
    if (st != WC_OK) return st;
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (mode != WC_WAVE && mode != WC_BLOCK) return run_sssp(ctx, g, nullptr, src, level, mode, tune, stream, stats);
    // wave and block modes: the recursion path (consolidated recursive calls)
    WC_HIP(hipSetDevice(ctx->device));
    Config cfg;
    st = resolve_tune(ctx, "bfs", mode, tune, 1 << 20, &cfg);
    if (st != WC_OK) return st;
    if (cfg.driver != 0) return fail(WC_EINVAL, "wc_bfs: drivers 2 and 3 are comparison variants of grid mode only");
    if (cfg.buffer_alloc != 0) return fail(WC_EINVAL, "wc_bfs: buffer_alloc does not apply to the recursion path");
    int overflowed = 0;
    st = run_bfs_rec(ctx, g, src, level, mode, cfg, stream, stats, &overflowed);
    if (st != WC_OK || !overflowed) return st;
    // the call list was too small: the frontier rounds recompute the levels
    st = run_sssp(ctx, g, nullptr, src, level, mode, tune, stream, stats);
    if (stats) stats->overflowed = 1;
    if (st == WC_OK && cfg.fail_on_overflow)
        return fail(WC_EOVERFLOW, "wc_bfs: the call list overflowed (buf_capacity too small)");
    return st;
}
