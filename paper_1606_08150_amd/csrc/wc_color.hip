// Graph coloring with workload consolidation (the GC benchmark of Sec. V, an
// irregular loop like Fig. 1(b)).
//
// Jones-Plassmann coloring of a symmetric graph: a vertex takes color r in the
// round after its last outranking neighbour was colored (r - 1), color 0 if no
// neighbour outranks it (larger priority, ties to the larger id).  This is the
// round-by-round definition (every uncolored vertex that outranks all of its
// uncolored neighbours takes the round's color) computed data-driven: wait[v]
// counts the outranking neighbours still uncolored; a vertex colored in round
// r loops over its neighbours and releases the ones it outranks, and a vertex
// whose count reaches zero joins the queue of round r + 1 with color r + 1.
// Every edge is visited once by the count pass and once by a release, instead
// of once per round.
//
// A queued vertex's release loop is the nested work; one with more than
// `threshold` neighbours is consolidated per mode:
//   wave  - the wave's ballot mask is the buffer; the wave walks each buffered
//           vertex's neighbours 64 at a time (no barrier).
//   block - thread-ordered LDS buffer; after the barrier the block walks the
//           concatenated neighbour ranges.
//   grid  - global buffer of (vertex, neighbour range) chunks drained by a
//           moldable grid after the kernel boundary, one wave per chunk.
//   flat  - every vertex walks all of its neighbours itself.
#include <algorithm>
#include <cstring>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

constexpr int kPad = 32;        // ring entries on separate 128-byte lines
constexpr int kUnroll = 4;      // neighbours in flight per lane

struct ColorArgs {
    const int *row_ptr;
    const int *col;
    const uint32_t *prio;
    int *color;       // -1 while uncolored
    int *wait;        // outranking neighbours not yet colored
    int *queue0;      // vertices colored in even rounds
    int *queue1;      // ... in odd rounds
    int *qtail;       // ring of 3 (stride kPad): size of the queue of round r
    int *chunk_tail;  // ring of 3 (stride kPad)
    int4 *chunks;     // (v, begin, end, prio[v])
    long long chunk_cap;
    int n;
    int threshold;
    int chunk;
    int *host_ring;
    DevStats *stats;
    int want_stats;
};

__device__ __forceinline__ bool above(uint32_t pu, int u, uint32_t pv, int v)
{
    return pu > pv || (pu == pv && u > v);
}

// v (priority pv, colored in round r) releases its neighbours e = first +
// k * stride < end that it outranks; a neighbour whose count reaches zero is
// appended to the next round's queue with color r + 1.  Every active lane of
// the wave calls this together (the appends are wave-aggregated); v, first,
// stride and end may differ per lane.  Returns the number of releases.
__device__ __forceinline__ int release_range(const ColorArgs &a, int v, uint32_t pv, int first, int stride, int end,
                                             int *next, int *next_tail, int color_next)
{
    int rel = 0;
    for (int e0 = first; e0 < end; e0 += kUnroll * stride) {
        int w[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int e = e0 + k * stride;
            w[k] = e < end ? a.col[e] : v;
        }
        uint32_t pw[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) pw[k] = w[k] != v ? a.prio[w[k]] : 0u;
        int old[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const bool out = w[k] != v && above(pv, v, pw[k], w[k]);
            old[k] = out ? atomic_add_dev(&a.wait[w[k]], -1) : 0;
            rel += out ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const bool ready = old[k] == 1;
            const int s = wave_reserve(ready, next_tail);
            if (ready) {
                next[s] = w[k];
                a.color[w[k]] = color_next;
            }
        }
    }
    return rel;
}

// One neighbour w of v (block-level drain, one edge per thread).
__device__ __forceinline__ int release_one(const ColorArgs &a, int v, uint32_t pv, int w, int *next, int *next_tail,
                                           int color_next)
{
    const bool out = w != v && above(pv, v, a.prio[w], w);
    const bool ready = out && atomic_add_dev(&a.wait[w], -1) == 1;
    const int s = wave_reserve(ready, next_tail);
    if (ready) {
        next[s] = w;
        a.color[w] = color_next;
    }
    return out ? 1 : 0;
}

template <int BLOCK>
struct ColorLds {
    int v[BLOCK];
    int beg[BLOCK];
    uint32_t p[BLOCK];
    int pre[BLOCK + 1];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
};

// Round r: thread i takes the i-th vertex of the round's queue (colored r).
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_round(ColorArgs a, int r)
{
    __shared__ ColorLds<BLOCK> sb;
    const int size = a.qtail[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.qtail[((r + 2) % 3) * kPad] = 0;
        a.chunk_tail[((r + 1) % 3) * kPad] = 0;
        store_system(&a.host_ring[r % kHostRing], size);
    }
    if (size == 0) return;
    const int *q = (r & 1) ? a.queue1 : a.queue0;
    int *next = (r & 1) ? a.queue0 : a.queue1;
    int *next_tail = &a.qtail[((r + 1) % 3) * kPad];
    const int lane = lane_id();
    StatAcc acc;
    for (int base = blockIdx.x * BLOCK; base < size; base += gridDim.x * BLOCK) {
        const int i = base + threadIdx.x;
        const bool member = i < size;
        int v = 0, beg = 0, end = 0;
        uint32_t pv = 0;
        if (member) {
            v = q[i];
            beg = a.row_ptr[v];
            end = a.row_ptr[v + 1];
            pv = a.prio[v];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        if (a.want_stats) {
            acc.edges += deg;
            acc.buffered += heavy ? deg : 0;
            acc.items += heavy ? 1 : 0;
            if (MODE == WC_WAVE && __ballot(heavy) && lane == 0) acc.dispatches += 1;
        }
        if (member && !heavy) acc.updates += release_range(a, v, pv, beg, 1, end, next, next_tail, r + 1);
        if constexpr (MODE == WC_WAVE) {
            uint64_t mask = __ballot(heavy);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                acc.updates_buffered += release_range(a, readlane(v, b), readlane_u(pv, b), readlane(beg, b) + lane,
                                                      kWave, readlane(end, b), next, next_tail, r + 1);
            }
        } else if constexpr (MODE == WC_BLOCK) {
            int k, off, nb, total;
            block_scan2<BLOCK>(heavy ? 1 : 0, heavy ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if (heavy) {
                sb.v[k] = v;
                sb.beg[k] = beg;
                sb.p[k] = pv;
                sb.pre[k] = off;
            }
            if (threadIdx.x == 0) {
                sb.pre[nb] = total;
                if (a.want_stats && nb) acc.dispatches += 1;
            }
            __syncthreads();
            int it = 0;
            for (int j = threadIdx.x; j < total; j += BLOCK) {
                while (it + 1 < nb && sb.pre[it + 1] <= j) ++it;
                const int w = a.col[sb.beg[it] + (j - sb.pre[it])];
                acc.updates_buffered += release_one(a, sb.v[it], sb.p[it], w, next, next_tail, r + 1);
            }
            __syncthreads();  // the LDS buffer is reused by the next window
        } else if constexpr (MODE == WC_GRID) {
            if (__syncthreads_or(heavy ? 1 : 0)) {
                const int nch = heavy ? (deg + a.chunk - 1) / a.chunk : 0;
                int excl, unused, tot, unused2;
                block_scan2<BLOCK>(nch, 0, sb.scan_tmp, excl, unused, tot, unused2);
                if (threadIdx.x == 0) sb.base = tot ? atomic_add_dev(&a.chunk_tail[(r % 3) * kPad], tot) : 0;
                __syncthreads();
                const long long slot = (long long)sb.base + excl;
                const bool fits = slot + nch <= a.chunk_cap;
                if (heavy) {
                    if (fits) {
                        for (int c = 0; c < nch; ++c) {
                            const int cb = beg + c * a.chunk;
                            a.chunks[slot + c] = make_int4(v, cb, min(end, cb + a.chunk), (int)pv);
                        }
                    } else {
                        // buffer full: the reserved slots below the capacity get
                        // empty ranges (the drain reads no stale chunk there) and
                        // this vertex is walked inline (fallback)
                        a.stats->overflowed = 1;
                        for (long long c = slot; c < slot + nch && c < a.chunk_cap; ++c)
                            a.chunks[c] = make_int4(v, 0, 0, 0);
                    }
                }
                if (heavy && !fits) acc.updates += release_range(a, v, pv, beg, 1, end, next, next_tail, r + 1);
                __syncthreads();  // sb.base is rewritten by the next window
            }
        }
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Consolidated child of grid mode: one wave per chunk.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_drain(ColorArgs a, int r)
{
    if (a.qtail[(r % 3) * kPad] == 0) return;
    const int tail = a.chunk_tail[(r % 3) * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    int *next = (r & 1) ? a.queue0 : a.queue1;
    int *next_tail = &a.qtail[((r + 1) % 3) * kPad];
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    StatAcc acc;
    if (a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0) acc.dispatches = 1;
    for (int c = gw; c < total; c += nw) {
        const int4 d = a.chunks[c];
        acc.updates_buffered += release_range(
            a, __builtin_amdgcn_readfirstlane(d.x), (uint32_t)__builtin_amdgcn_readfirstlane(d.w),
            __builtin_amdgcn_readfirstlane(d.y) + lane_id(), kWave, __builtin_amdgcn_readfirstlane(d.z), next,
            next_tail, r + 1);
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Clears the rings before the count pass appends to the first queue.
__global__ void color_reset(ColorArgs a)
{
    if (threadIdx.x < 3) {
        a.qtail[threadIdx.x * kPad] = 0;
        a.chunk_tail[threadIdx.x * kPad] = 0;
    }
}

// Neighbours e = first + k * stride < end of v (priority pv) that outrank v.
__device__ __forceinline__ int count_range(const ColorArgs &a, int v, uint32_t pv, int first, int stride, int end)
{
    int cnt = 0;
    for (int e0 = first; e0 < end; e0 += kUnroll * stride) {
        int u[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int e = e0 + k * stride;
            u[k] = e < end ? a.col[e] : v;
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cnt += u[k] != v && above(a.prio[u[k]], u[k], pv, v) ? 1 : 0;
    }
    return cnt;
}

template <int BLOCK>
struct CountLds {
    int v[BLOCK];
    int beg[BLOCK];
    uint32_t p[BLOCK];
    int pre[BLOCK + 1];
    int cnt[BLOCK];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
};

// Count pass, the first irregular loop: wait[v] = neighbours that outrank v.
// A row with more than `threshold` entries is consolidated per mode (grid:
// its chunks are counted by color_count_drain, which adds to wait[v] = 0).
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_count(ColorArgs a)
{
    __shared__ CountLds<BLOCK> sb;
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {
        const int v = base + threadIdx.x;
        const bool member = v < a.n;
        int beg = 0, end = 0;
        uint32_t pv = 0;
        if (member) {
            beg = a.row_ptr[v];
            end = a.row_ptr[v + 1];
            pv = a.prio[v];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        int cnt = 0;
        if (member && !heavy) cnt = count_range(a, v, pv, beg, 1, end);
        if constexpr (MODE == WC_WAVE) {
            uint64_t mask = __ballot(heavy);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int c = wave_sum_i(count_range(a, readlane(v, b), readlane_u(pv, b), readlane(beg, b) + lane,
                                                     kWave, readlane(end, b)));
                if (lane == b) cnt = c;
            }
        } else if constexpr (MODE == WC_BLOCK) {
            int k, off, nb, total;
            block_scan2<BLOCK>(heavy ? 1 : 0, heavy ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if (heavy) {
                sb.v[k] = v;
                sb.beg[k] = beg;
                sb.p[k] = pv;
                sb.pre[k] = off;
                sb.cnt[k] = 0;
            }
            if (threadIdx.x == 0) sb.pre[nb] = total;
            __syncthreads();
            int it = 0;
            for (int j = threadIdx.x; j < total; j += BLOCK) {
                while (it + 1 < nb && sb.pre[it + 1] <= j) ++it;
                const int u = a.col[sb.beg[it] + (j - sb.pre[it])];
                if (u != sb.v[it] && above(a.prio[u], u, sb.p[it], sb.v[it])) atomicAdd(&sb.cnt[it], 1);
            }
            __syncthreads();
            if (heavy) cnt = sb.cnt[k];
            __syncthreads();  // the LDS buffer is reused by the next window
        } else if constexpr (MODE == WC_GRID) {
            if (__syncthreads_or(heavy ? 1 : 0)) {
                const int nch = heavy ? (deg + a.chunk - 1) / a.chunk : 0;
                int excl, unused, tot, unused2;
                block_scan2<BLOCK>(nch, 0, sb.scan_tmp, excl, unused, tot, unused2);
                if (threadIdx.x == 0) sb.base = tot ? atomic_add_dev(&a.chunk_tail[2 * kPad], tot) : 0;
                __syncthreads();
                const long long slot = (long long)sb.base + excl;
                const bool fits = slot + nch <= a.chunk_cap;
                if (heavy) {
                    if (fits) {
                        for (int c = 0; c < nch; ++c) {
                            const int cb = beg + c * a.chunk;
                            a.chunks[slot + c] = make_int4(v, cb, min(end, cb + a.chunk), (int)pv);
                        }
                    } else {
                        a.stats->overflowed = 1;
                        for (long long c = slot; c < slot + nch && c < a.chunk_cap; ++c)
                            a.chunks[c] = make_int4(v, 0, 0, 0);
                        cnt = count_range(a, v, pv, beg, 1, end);  // fallback: counted inline
                    }
                }
                __syncthreads();  // sb.base is rewritten by the next window
            }
        }
        if (member) a.wait[v] = cnt;
    }
}

// Grid mode: one wave per chunk of a long row adds its count to wait[v].
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_count_drain(ColorArgs a)
{
    const int tail = a.chunk_tail[2 * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    for (int c = gw; c < total; c += nw) {
        const int4 d = a.chunks[c];
        const int v = __builtin_amdgcn_readfirstlane(d.x);
        const int cnt = wave_sum_i(count_range(a, v, (uint32_t)__builtin_amdgcn_readfirstlane(d.w),
                                               __builtin_amdgcn_readfirstlane(d.y) + lane_id(), kWave,
                                               __builtin_amdgcn_readfirstlane(d.z)));
        if (lane_id() == 0 && cnt) (void)atomic_add_dev(&a.wait[v], cnt);
    }
}

// Vertices that no neighbour outranks take color 0 and form the queue of
// round 0; the others start uncolored.  One queue reservation per block step.
constexpr int kSeedBlock = 256;
__global__ __launch_bounds__(kSeedBlock) void color_seed(ColorArgs a)
{
    __shared__ int scan_tmp[2 * (kSeedBlock / kWave)];
    __shared__ int s_base;
    for (int base = blockIdx.x * kSeedBlock; base < a.n; base += gridDim.x * kSeedBlock) {
        const int v = base + threadIdx.x;
        const bool member = v < a.n;
        const bool first = member && a.wait[v] == 0;
        if (member) a.color[v] = first ? 0 : -1;
        int k, unused, tot, unused2;
        block_scan2<kSeedBlock>(first ? 1 : 0, 0, scan_tmp, k, unused, tot, unused2);
        if (threadIdx.x == 0 && tot) s_base = atomic_add_dev(&a.qtail[0], tot);
        __syncthreads();
        if (first) a.queue0[s_base + k] = v;
        __syncthreads();  // s_base is rewritten by the next step
    }
}

struct ColorKernels {
    const void *round, *drain, *count, *count_drain;
};

template <int BLOCK>
ColorKernels pick_block(wc_mode mode)
{
    ColorKernels k{nullptr, reinterpret_cast<const void *>(&color_drain<BLOCK>), nullptr,
                   reinterpret_cast<const void *>(&color_count_drain<BLOCK>)};
    switch (mode) {
    case WC_FLAT:
        k.round = reinterpret_cast<const void *>(&color_round<WC_FLAT, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_FLAT, BLOCK>);
        break;
    case WC_WAVE:
        k.round = reinterpret_cast<const void *>(&color_round<WC_WAVE, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_WAVE, BLOCK>);
        break;
    case WC_BLOCK:
        k.round = reinterpret_cast<const void *>(&color_round<WC_BLOCK, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_BLOCK, BLOCK>);
        break;
    default:
        k.round = reinterpret_cast<const void *>(&color_round<WC_GRID, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_GRID, BLOCK>);
        break;
    }
    return k;
}

ColorKernels pick(wc_mode mode, int block)
{
    switch (block) {
    case 64: return pick_block<64>(mode);
    case 128: return pick_block<128>(mode);
    case 512: return pick_block<512>(mode);
    case 1024: return pick_block<1024>(mode);
    default: return pick_block<256>(mode);
    }
}

}  // namespace
}  // namespace wc

using namespace wc;

extern "C" wc_status wc_color(wc_ctx *ctx, const wc_csr *g, const uint32_t *prio, int32_t *color, wc_mode mode,
                              const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !g) return fail(WC_EINVAL, "wc_color: NULL context or graph");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_color: bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, "wc_color: negative size");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (!g->row_ptr || !prio || !color || (g->m > 0 && !g->col)) return fail(WC_EINVAL, "wc_color: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    ColorKernels ks = pick(mode, block);
    int resident = resident_blocks(ctx, ks.round, block);
    Config cfg;
    wc_status st = resolve_tune(ctx, "color", mode, tune, resident, &cfg);
    if (st != WC_OK) return st;
    if (cfg.driver != 0) return fail(WC_EINVAL, "wc_color: only the relaunch driver (driver = 0) exists");
    if (cfg.block != block) {
        ks = pick(mode, cfg.block);
        resident = resident_blocks(ctx, ks.round, cfg.block);
    }
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    const bool grid_mode = mode == WC_GRID;
    // every vertex has ceil(deg / chunk) <= deg / chunk + 1 chunks in the one
    // round that colors it, so n + m / chunk + 1 entries never overflow
    const long long cap_full = n + m / chunk + 1;
    const long long cap = grid_mode ? (cfg.buf_capacity > 0 ? std::min(cfg.buf_capacity, cap_full) : cap_full) : 1;
    const size_t need = 3 * padded(n * 4) + 2 * padded(3 * kPad * 4) + padded(cap * 16);
    st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    ColorArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.prio = prio;
    a.color = color;
    a.wait = pool_take<int>(ctx, n);
    a.queue0 = pool_take<int>(ctx, n);
    a.queue1 = pool_take<int>(ctx, n);
    a.qtail = pool_take<int>(ctx, 3 * kPad);
    a.chunk_tail = pool_take<int>(ctx, 3 * kPad);
    a.chunks = pool_take<int4>(ctx, cap);
    a.chunk_cap = cap;
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.chunk = chunk;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    const int grid = std::max(1, std::min<int>(std::min(cfg.grid, resident), (int)((n + cfg.block - 1) / cfg.block)));
    const int dgrid = std::max(1, std::min(cfg.grid, resident));
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    {
        void *args[] = {&a};
        st = launch(ctx, "color_reset", reinterpret_cast<const void *>(&color_reset), dim3(1), dim3(64), args,
                    stream);
        if (st == WC_OK) st = launch(ctx, "color_count", ks.count, dim3(grid), dim3(cfg.block), args, stream);
        if (st == WC_OK && grid_mode)
            st = launch(ctx, "color_count_drain", ks.count_drain, dim3(dgrid), dim3(cfg.block), args, stream);
        const int sg = (int)std::min<long long>((n + kSeedBlock - 1) / kSeedBlock, 4096);
        if (st == WC_OK)
            st = launch(ctx, "color_seed", reinterpret_cast<const void *>(&color_seed), dim3(sg), dim3(kSeedBlock),
                        args, stream);
        if (st != WC_OK) return st;
    }
    static const char *names[] = {"color_round_flat", "color_round_wave", "color_round_block", "color_round_grid"};
    // relaunch driver: rounds kept in flight (each publishes its queue size);
    // the first empty round ends the loop
    const int window = 4;
    int rounds = 0, launched = 0;
    long long colored = 0;
    for (;;) {
        while (launched < rounds + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, names[mode], ks.round, dim3(grid), dim3(cfg.block), args, stream);
            if (st == WC_OK && grid_mode)
                st = launch(ctx, "color_drain", ks.drain, dim3(dgrid), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            ++launched;
        }
        int c = 0;
        st = wait_round_count(ctx, rounds, &c);
        if (st != WC_OK) return st;
        if (c == 0) break;
        colored += c;
        ++rounds;
        if (colored > n) return fail(WC_EINVAL, "wc_color: more queued vertices than vertices");
    }
    st = end_call(ctx, stream, stats, rounds, cfg.fail_on_overflow);
    if (st != WC_OK) return st;
    if (colored != n)
        return fail(WC_EINVAL, "wc_color: some vertices never became ready (the graph is not symmetric)");
    return WC_OK;
}
