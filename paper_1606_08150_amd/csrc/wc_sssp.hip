// SSSP with workload consolidation (irregular loop of Fig. 1(b)).
//
// Frontier-driven rounds: round r expands every vertex whose distance improved
// in round r-1.  A frontier vertex is one parent work item; its prework reads
// its CSR range and current distance, and the condition of Fig. 1(b) compares
// its out-degree with the threshold.  A light vertex relaxes its edges inline
// ("work"); a heavy one is inserted into the consolidation buffer of its mode
// and relaxed by the consolidated child ("process_neighbors"):
//   wave  - the wave's ballot mask is the buffer; the whole wave then relaxes
//           each buffered vertex's edges, 64 lanes side by side (no barrier).
//   block - thread-ordered LDS buffer; after the workgroup barrier the block
//           relaxes the concatenated edge ranges of all buffered vertices, each
//           thread taking every BLOCK-th edge (a multi-thread child wrapped in a
//           loop over the buffer, Sec. IV.C, load-balanced over items).
//   grid  - global buffer of (vertex, edge range) chunks of 64 * items_per_lane
//           edges, appended with one atomic per wave; after the grid-wide
//           barrier a moldable grid drains all chunks, one wave per chunk.
//   flat  - every vertex relaxes all of its edges itself.
// Relaxation: nd = dist[u] + w; atomicMin on dist[v]; an improved vertex is
// appended once per round to the next frontier (per-vertex round stamp).
// The distances reached are the unique shortest-path distances, so every mode
// and schedule yields identical results.
#include <cstring>
#include <algorithm>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"

namespace wc {
namespace {

struct SsspArgs {
    const int *row_ptr;
    const int *col;
    const uint32_t *w;
    uint32_t *dist;
    int *stamp;
    int *frontier0;
    int *frontier1;
    int *counts;      // ring of 3 frontier sizes
    int *chunk_tail;  // ring of 3 grid-buffer tails
    int4 *chunks;     // grid consolidation buffer: (u, begin, end, 0)
    long long chunk_cap;
    int n;
    int threshold;
    int chunk;
    int *host_ring;
    DevStats *stats;
    int want_stats;
    GridBarrier *bar;
    int bar_blocks;
};

__device__ __forceinline__ int *frontier_of(const SsspArgs &a, int r) { return (r & 1) ? a.frontier1 : a.frontier0; }

// One relaxation; true when v must join the next frontier (first improvement
// of v in this round).
__device__ __forceinline__ bool relax_one(const SsspArgs &a, int v, uint32_t nd, int next)
{
    if (nd >= a.dist[v]) return false;  // a stale read is only ever too high
    uint32_t old = atomic_min_dev(&a.dist[v], nd);
    if (nd >= old) return false;
    return atomic_exch_dev(&a.stamp[v], next) != next;
}

__device__ __forceinline__ uint32_t add_sat(uint32_t du, uint32_t w)
{
    uint32_t s = du + w;
    return s < du ? kInf : s;
}

// Inline "work" of Fig. 1(b): the lane relaxes edges [beg, end) of its vertex.
__device__ __forceinline__ void relax_lane(const SsspArgs &a, int beg, int end, uint32_t du, int *fout,
                                           int *cnt, int next)
{
    for (int e = beg; e < end; ++e) {
        int v = a.col[e];
        bool enq = relax_one(a, v, add_sat(du, a.w[e]), next);
        int slot = wave_reserve(enq, cnt);
        if (enq) fout[slot] = v;
    }
}

// The wave cooperatively relaxes edges [beg, end) of one vertex (uniform arguments).
__device__ __forceinline__ void relax_wave(const SsspArgs &a, int beg, int end, uint32_t du, int *fout, int *cnt,
                                           int next)
{
    for (int e = beg + lane_id(); e < end; e += kWave) {
        int v = a.col[e];
        bool enq = relax_one(a, v, add_sat(du, a.w[e]), next);
        int slot = wave_reserve(enq, cnt);
        if (enq) fout[slot] = v;
    }
}

template <int BLOCK>
struct BlockBuf {
    int beg[BLOCK];
    uint32_t du[BLOCK];
    int pre[BLOCK + 1];
    int scan_tmp[2 * (BLOCK / kWave)];
};

// Parent phase of round r over the whole frontier (grid-stride windows of
// BLOCK items; every thread of a block runs the same number of windows).
template <int MODE, int BLOCK>
__device__ void parent_phase(const SsspArgs &a, int r, int count)
{
    const int *fin = frontier_of(a, r);
    int *fout = frontier_of(a, r + 1);
    int *cnt = &a.counts[(r + 1) % 3];
    const int next = r + 1;
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK; base < count; base += gridDim.x * BLOCK) {
        const int i = base + threadIdx.x;
        const bool valid = i < count;
        int u = 0, beg = 0, end = 0;
        uint32_t du = 0;
        if (valid) {
            u = fin[i];
            beg = a.row_ptr[u];
            end = a.row_ptr[u + 1];
            du = a.dist[u];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        if (a.want_stats) {
            int s = wave_sum_i(deg);
            uint64_t hm = __ballot(heavy);
            if (lane == 0) {
                atomic_add_dev(&a.stats->edges_processed, (unsigned long long)s);
                atomic_add_dev(&a.stats->items_buffered, (unsigned long long)__builtin_popcountll(hm));
                if (MODE == WC_WAVE && hm) atomic_add_dev(&a.stats->dispatches, 1ull);
            }
        }
        // work: light items relax inline
        relax_lane(a, beg, heavy ? beg : end, du, fout, cnt, next);

        if constexpr (MODE == WC_WAVE) {
            // insert_buffer = ballot; the mask is the wave's buffer; no barrier needed
            uint64_t mask = __ballot(heavy);
            while (mask) {
                int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                relax_wave(a, readlane(beg, b), readlane(end, b), readlane_u(du, b), fout, cnt, next);
            }
        } else if constexpr (MODE == WC_BLOCK) {
            __shared__ BlockBuf<BLOCK> sb;
            int k, off, nb, total;
            block_scan2<BLOCK>(heavy ? 1 : 0, heavy ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if (heavy) {
                sb.beg[k] = beg;
                sb.du[k] = du;
                sb.pre[k] = off;
            }
            if (threadIdx.x == 0) {
                sb.pre[nb] = total;
                if (a.want_stats && nb) atomic_add_dev(&a.stats->dispatches, 1ull);
            }
            __syncthreads();  // the "synchronize" between inserts and the child
            if (nb) {
                int it = 0;
                for (int j = threadIdx.x; j < total; j += BLOCK) {
                    while (it + 1 < nb && sb.pre[it + 1] <= j) ++it;
                    int e = sb.beg[it] + (j - sb.pre[it]);
                    int v = a.col[e];
                    bool enq = relax_one(a, v, add_sat(sb.du[it], a.w[e]), next);
                    int slot = wave_reserve(enq, cnt);
                    if (enq) fout[slot] = v;
                }
            }
            __syncthreads();  // LDS buffer is reused by the next window
        } else if constexpr (MODE == WC_GRID) {
            const int nch = heavy ? (deg + a.chunk - 1) / a.chunk : 0;
            const int slot = wave_reserve_n(nch, &a.chunk_tail[r % 3]);
            if (heavy) {
                for (int c = 0; c < nch; ++c) {
                    int cb = beg + c * a.chunk;
                    int ce = min(end, cb + a.chunk);
                    if ((long long)slot + c < a.chunk_cap) {
                        a.chunks[slot + c] = make_int4(u, cb, ce, 0);
                    } else {
                        // buffer full: this chunk is processed inline (fallback)
                        a.stats->overflowed = 1;
                        relax_lane(a, cb, ce, du, fout, cnt, next);
                    }
                }
            }
        }
    }
}

// Consolidated child of grid-level consolidation: one wave per chunk, chunks
// fetched grid-stride until the buffer is exhausted (moldable).
template <int BLOCK>
__device__ void drain_phase(const SsspArgs &a, int r)
{
    const int tail = a.chunk_tail[r % 3];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    int *fout = frontier_of(a, r + 1);
    int *cnt = &a.counts[(r + 1) % 3];
    const int next = r + 1;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    if (a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0)
        atomic_add_dev(&a.stats->dispatches, 1ull);
    for (int c = gw; c < total; c += nw) {
        int4 d = a.chunks[c];
        int u = __builtin_amdgcn_readfirstlane(d.x);
        int cb = __builtin_amdgcn_readfirstlane(d.y);
        int ce = __builtin_amdgcn_readfirstlane(d.z);
        uint32_t du = a.dist[u];
        relax_wave(a, cb, ce, du, fout, cnt, next);
    }
}

__global__ void sssp_init(SsspArgs a, int src)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < a.n; i += gridDim.x * blockDim.x) {
        a.dist[i] = i == src ? 0u : kInf;
        a.stamp[i] = i == src ? 0 : -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.frontier0[0] = src;
        a.counts[0] = 1;
        a.counts[1] = 0;
        a.counts[2] = 0;
        a.chunk_tail[0] = a.chunk_tail[1] = a.chunk_tail[2] = 0;
        a.bar->count = a.bar_blocks;
        a.bar->generation = 0;
    }
}

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_round(SsspArgs a, int r)
{
    const int count = a.counts[r % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.counts[(r + 2) % 3] = 0;
        if (MODE == WC_GRID) a.chunk_tail[(r + 1) % 3] = 0;
        store_system(&a.host_ring[r % kHostRing], count);
    }
    if (count == 0) return;
    parent_phase<MODE, BLOCK>(a, r, count);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_drain(SsspArgs a, int r)
{
    if (a.counts[r % 3] == 0) return;
    drain_phase<BLOCK>(a, r);
}

// Persistent driver: every round in one co-resident launch; the grid barrier
// of Sec. IV.E separates inserts from the drain and one round from the next.
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_persistent(SsspArgs a, int max_rounds)
{
    const int nb = gridDim.x;
    int r = 0;
    for (; r < max_rounds; ++r) {
        const int count = atomic_load_dev(&a.counts[r % 3]);
        if (count == 0) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.counts[(r + 2) % 3] = 0;
            if (MODE == WC_GRID) a.chunk_tail[(r + 1) % 3] = 0;
        }
        parent_phase<MODE, BLOCK>(a, r, count);
        if (!grid_barrier(a.bar, nb)) {
            a.stats->timed_out = 1;
            return;
        }
        if constexpr (MODE == WC_GRID) {
            drain_phase<BLOCK>(a, r);
            if (!grid_barrier(a.bar, nb)) {
                a.stats->timed_out = 1;
                return;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.stats->rounds = r;
}

// ---- host side --------------------------------------------------------------------------------

template <int MODE, int BLOCK>
struct SsspKernels {
    static const void *round() { return reinterpret_cast<const void *>(&sssp_round<MODE, BLOCK>); }
    static const void *drain() { return reinterpret_cast<const void *>(&sssp_drain<BLOCK>); }
    static const void *persistent() { return reinterpret_cast<const void *>(&sssp_persistent<MODE, BLOCK>); }
};

struct KernelSet {
    const void *round, *drain, *persistent;
};

template <int BLOCK>
KernelSet pick_block(wc_mode mode)
{
    switch (mode) {
    case WC_FLAT: return {SsspKernels<WC_FLAT, BLOCK>::round(), nullptr, SsspKernels<WC_FLAT, BLOCK>::persistent()};
    case WC_WAVE: return {SsspKernels<WC_WAVE, BLOCK>::round(), nullptr, SsspKernels<WC_WAVE, BLOCK>::persistent()};
    case WC_BLOCK:
        return {SsspKernels<WC_BLOCK, BLOCK>::round(), nullptr, SsspKernels<WC_BLOCK, BLOCK>::persistent()};
    default:
        return {SsspKernels<WC_GRID, BLOCK>::round(), SsspKernels<WC_GRID, BLOCK>::drain(),
                SsspKernels<WC_GRID, BLOCK>::persistent()};
    }
}

const char *round_name(wc_mode mode)
{
    static const char *names[] = {"sssp_round_flat", "sssp_round_wave", "sssp_round_block", "sssp_round_grid"};
    return names[mode];
}

KernelSet pick(wc_mode mode, int block)
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

extern "C" wc_status wc_sssp(wc_ctx *ctx, const wc_csr *g, const uint32_t *w, int32_t src, uint32_t *dist,
                             wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !g) return fail(WC_EINVAL, "wc_sssp: NULL context or graph");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_sssp: bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, "wc_sssp: negative size");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (src < 0 || src >= g->n) return fail(WC_EINVAL, "wc_sssp: source out of range");
    if (!g->row_ptr || !dist || (g->m > 0 && (!g->col || !w))) return fail(WC_EINVAL, "wc_sssp: NULL array");
    WC_HIP(hipSetDevice(ctx->device));

    Config cfg;
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    KernelSet ks = pick(mode, block);
    int resident = resident_blocks(ctx, ks.persistent, block);
    wc_status st = resolve_tune(ctx, "sssp", mode, tune, resident, &cfg);
    if (st != WC_OK) return st;
    if (cfg.block != block) {
        ks = pick(mode, cfg.block);
        resident = resident_blocks(ctx, ks.persistent, cfg.block);
    }
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    // Grid buffer: every frontier vertex (at most n per round) yields at most
    // ceil(deg / chunk) chunks, so n + m / chunk + 1 entries never overflow.
    long long cap_full = n + m / chunk + 1;
    long long cap = mode == WC_GRID ? (cfg.buf_capacity > 0 ? std::min(cfg.buf_capacity, cap_full) : cap_full) : 1;
    size_t need = padded(n * 4) * 3 + padded(3 * 4) * 2 + padded(cap * 16) + padded(sizeof(GridBarrier));
    st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    SsspArgs a;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.w = w;
    a.dist = dist;
    a.stamp = pool_take<int>(ctx, n);
    a.frontier0 = pool_take<int>(ctx, n);
    a.frontier1 = pool_take<int>(ctx, n);
    a.counts = pool_take<int>(ctx, 3);
    a.chunk_tail = pool_take<int>(ctx, 3);
    a.chunks = pool_take<int4>(ctx, cap);
    a.bar = pool_take<GridBarrier>(ctx, 1);
    a.chunk_cap = cap;
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.chunk = chunk;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;

    const int grid = std::max(1, std::min(cfg.grid, resident));
    a.bar_blocks = grid;  // the barrier counter starts at the number of blocks
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    int init_grid = (int)std::min<long long>((n + 255) / 256, 4096);
    {
        void *args[] = {&a, &src};
        st = launch(ctx, "sssp_init", reinterpret_cast<const void *>(&sssp_init), dim3(init_grid), dim3(256), args,
                    stream);
        if (st != WC_OK) return st;
    }

    int rounds = 0;
    if (cfg.driver == 1) {
        return fail(WC_EINVAL, "the persistent driver (driver = 1) is disabled: use the relaunch driver");
        int max_rounds = (int)std::min<long long>(n + 1, 0x7fffffff);
        void *args[] = {&a, &max_rounds};
        WC_HIP(hipLaunchCooperativeKernel(ks.persistent, dim3(grid), dim3(cfg.block), args, 0, stream));
        st = end_call(ctx, stream, stats, -1, cfg.fail_on_overflow);
        if (stats && st == WC_OK) {
            int r = 0;
            WC_HIP(hipMemcpy(&r, &ctx->dstats->rounds, sizeof(int), hipMemcpyDeviceToHost));
            stats->rounds = r;
        }
        return st;
    }
    // Relaunch driver: keep `window` rounds in flight; each round kernel
    // publishes its input size to pinned host memory, and the first empty round
    // ends the loop (later rounds already enqueued find empty frontiers).
    const int window = 4;
    int launched = 0;
    for (;;) {
        while (launched < rounds + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, round_name(mode), ks.round, dim3(grid), dim3(cfg.block), args, stream);
            if (st == WC_OK && mode == WC_GRID)
                st = launch(ctx, "sssp_drain", ks.drain, dim3(grid), dim3(cfg.block), args, stream);
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
