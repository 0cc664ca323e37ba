// SpMV with workload consolidation (irregular loop over CSR rows).
//
// One parent work item per row.  Prework reads the row's range; a row with
// more than `threshold` nonzeros is inserted into the consolidation buffer of
// its mode, a lighter row is summed inline by its lane ("work").
//   wave  - ballot-mask buffer; the wave sums each buffered row, lane l taking
//           elements l, l+64, ..., then a fixed butterfly reduction.
//   block - thread-ordered LDS buffer, then the workgroup barrier.  Rows longer
//           than BLOCK * items_per_lane are summed by the whole block (fixed
//           block reduction); the others are shared out to the block's waves.
//   grid  - global buffer of row chunks of 64 * items_per_lane nonzeros; after
//           the grid-wide barrier one wave sums each chunk.  A row split into
//           several chunks also gets an entry in a second buffer, and its chunk
//           partials are combined in chunk order (deterministic).
//   flat  - every row is summed by its own lane.
// All sums use fp32 fused multiply-adds in a fixed order per mode and tune, so
// results are bitwise reproducible; each stays within 1e-5 of the row's
// magnitude sum of the exact product.
#include <cstring>
#include <algorithm>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"

namespace wc {
namespace {

struct SpmvArgs {
    const int *row_ptr;
    const int *col;
    const float *val;
    const float *x;
    float *y;
    int n;
    int threshold;
    int chunk;
    int big;           // block mode: rows longer than this use the whole block
    int4 *chunks;      // (row, begin, end, 1 if the row has several chunks)
    long long chunk_cap;
    int *chunk_tail;
    int4 *multi;       // (row, first chunk, chunk count, 0)
    int *multi_tail;
    float *partials;   // one per chunk slot
    DevStats *stats;
    int want_stats;
};

__device__ __forceinline__ float dot_lane(const SpmvArgs &a, int beg, int end)
{
    float s = 0.f;
    for (int e = beg; e < end; ++e) s = fmaf(a.val[e], a.x[a.col[e]], s);
    return s;
}

// Whole-wave dot product of [beg, end) (uniform arguments); every lane gets the sum.
__device__ __forceinline__ float dot_wave(const SpmvArgs &a, int beg, int end)
{
    float s = 0.f;
    for (int e = beg + lane_id(); e < end; e += kWave) s = fmaf(a.val[e], a.x[a.col[e]], s);
    return wave_sum(s);
}

template <int BLOCK>
struct SpmvBlockBuf {
    int row[BLOCK];
    int beg[BLOCK];
    int end[BLOCK];
    int scan_tmp[2 * (BLOCK / kWave)];
    float red[BLOCK / kWave];
};

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_parent(SpmvArgs a)
{
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {
        const int r = base + threadIdx.x;
        const bool valid = r < a.n;
        int beg = 0, end = 0;
        if (valid) {
            beg = a.row_ptr[r];
            end = a.row_ptr[r + 1];
        }
        const int len = end - beg;
        const bool heavy = MODE != WC_FLAT && len > a.threshold;
        if (a.want_stats) {
            int s = wave_sum_i(len);
            uint64_t hm = __ballot(heavy);
            if (lane == 0) {
                atomic_add_dev(&a.stats->edges_processed, (unsigned long long)s);
                atomic_add_dev(&a.stats->items_buffered, (unsigned long long)__builtin_popcountll(hm));
                if (MODE == WC_WAVE && hm) atomic_add_dev(&a.stats->dispatches, 1ull);
            }
        }
        if (valid && !heavy) a.y[r] = dot_lane(a, beg, end);

        if constexpr (MODE == WC_WAVE) {
            uint64_t mask = __ballot(heavy);
            while (mask) {
                int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                float s = dot_wave(a, readlane(beg, b), readlane(end, b));
                if (lane == 0) a.y[base + (threadIdx.x & ~(kWave - 1)) + b] = s;
            }
        } else if constexpr (MODE == WC_BLOCK) {
            __shared__ SpmvBlockBuf<BLOCK> sb;
            constexpr int NW = BLOCK / kWave;
            int k, dummy, nb, dummy_total;
            block_scan2<BLOCK>(heavy ? 1 : 0, 0, sb.scan_tmp, k, dummy, nb, dummy_total);
            if (heavy) {
                sb.row[k] = r;
                sb.beg[k] = beg;
                sb.end[k] = end;
            }
            if (threadIdx.x == 0 && a.want_stats && nb) atomic_add_dev(&a.stats->dispatches, 1ull);
            __syncthreads();  // the "synchronize" between inserts and the child
            // rows too long for one wave: the whole block, one row at a time
            for (int it = 0; it < nb; ++it) {
                const int rb = sb.beg[it], re = sb.end[it];
                if (re - rb <= a.big) continue;
                float s = 0.f;
                for (int e = rb + (int)threadIdx.x; e < re; e += BLOCK) s = fmaf(a.val[e], a.x[a.col[e]], s);
                s = block_sum<BLOCK>(s, sb.red);
                if (threadIdx.x == 0) a.y[sb.row[it]] = s;
            }
            // the rest: one wave per row, rows dealt round-robin to the waves
            const int wid = threadIdx.x / kWave;
            for (int it = wid; it < nb; it += NW) {
                const int rb = sb.beg[it], re = sb.end[it];
                if (re - rb > a.big) continue;
                float s = dot_wave(a, rb, re);
                if (lane == 0) a.y[sb.row[it]] = s;
            }
            __syncthreads();  // LDS buffer is reused by the next window
        } else if constexpr (MODE == WC_GRID) {
            const int nch = heavy ? (len + a.chunk - 1) / a.chunk : 0;
            const int slot = wave_reserve_n(nch, a.chunk_tail);
            const bool fits = heavy && (long long)slot + nch <= a.chunk_cap;
            const int mslot = wave_reserve(fits && nch > 1, a.multi_tail);
            if (heavy) {
                if (fits) {
                    for (int c = 0; c < nch; ++c) {
                        int cb = beg + c * a.chunk;
                        a.chunks[slot + c] = make_int4(r, cb, min(end, cb + a.chunk), nch > 1 ? 1 : 0);
                    }
                    if (nch > 1) a.multi[mslot] = make_int4(r, slot, nch, 0);
                } else {
                    // buffer full: mark the reserved slots that exist as empty and
                    // sum the row inline (fallback)
                    for (int c = 0; c < nch; ++c)
                        if ((long long)slot + c < a.chunk_cap) a.chunks[slot + c] = make_int4(-1, 0, 0, 0);
                    a.stats->overflowed = 1;
                    a.y[r] = dot_lane(a, beg, end);
                }
            }
        }
    }
}

// Consolidated child of grid-level consolidation: one wave per chunk.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_drain(SpmvArgs a)
{
    const int tail = *a.chunk_tail;
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    if (a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0) atomic_add_dev(&a.stats->dispatches, 1ull);
    for (int c = gw; c < total; c += nw) {
        int4 d = a.chunks[c];
        int row = __builtin_amdgcn_readfirstlane(d.x);
        if (row < 0) continue;
        float s = dot_wave(a, __builtin_amdgcn_readfirstlane(d.y), __builtin_amdgcn_readfirstlane(d.z));
        if (lane_id() == 0) {
            if (d.w) a.partials[c] = s;
            else a.y[row] = s;
        }
    }
}

// Post-work of split rows: the chunk partials of each row, summed in chunk order.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_combine(SpmvArgs a)
{
    const int total = *a.multi_tail;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    for (int i = gw; i < total; i += nw) {
        int4 d = a.multi[i];
        int first = __builtin_amdgcn_readfirstlane(d.y), cnt = __builtin_amdgcn_readfirstlane(d.z);
        float s = 0.f;
        for (int c = lane_id(); c < cnt; c += kWave) s += a.partials[first + c];
        s = wave_sum(s);
        if (lane_id() == 0) a.y[d.x] = s;
    }
}

__global__ void spmv_reset(SpmvArgs a)
{
    if (threadIdx.x == 0) {
        *a.chunk_tail = 0;
        *a.multi_tail = 0;
    }
}

struct SpmvKernels {
    const void *parent, *drain, *combine;
};

template <int BLOCK>
SpmvKernels pick_block(wc_mode mode)
{
    SpmvKernels k{nullptr, reinterpret_cast<const void *>(&spmv_drain<BLOCK>),
                  reinterpret_cast<const void *>(&spmv_combine<BLOCK>)};
    switch (mode) {
    case WC_FLAT: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_FLAT, BLOCK>); break;
    case WC_WAVE: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_WAVE, BLOCK>); break;
    case WC_BLOCK: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_BLOCK, BLOCK>); break;
    default: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_GRID, BLOCK>); break;
    }
    return k;
}

SpmvKernels pick(wc_mode mode, int block)
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

extern "C" wc_status wc_spmv(wc_ctx *ctx, const wc_csr *g, const float *val, const float *x, float *y, wc_mode mode,
                             const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !g) return fail(WC_EINVAL, "wc_spmv: NULL context or matrix");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_spmv: bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, "wc_spmv: negative size");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (!g->row_ptr || !x || !y || (g->m > 0 && (!g->col || !val))) return fail(WC_EINVAL, "wc_spmv: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    SpmvKernels ks = pick(mode, block);
    int resident = resident_blocks(ctx, ks.parent, block);
    Config cfg;
    wc_status st = resolve_tune(ctx, "spmv", mode, tune, resident, &cfg);
    if (st != WC_OK) return st;
    if (cfg.block != block) {
        ks = pick(mode, cfg.block);
        resident = resident_blocks(ctx, ks.parent, cfg.block);
    }
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    long long cap_full = n + m / chunk + 1;
    long long cap = mode == WC_GRID ? (cfg.buf_capacity > 0 ? std::min(cfg.buf_capacity, cap_full) : cap_full) : 1;
    long long mcap = mode == WC_GRID ? cap / 2 + 1 : 1;
    size_t need = padded(cap * 16) + padded(cap * 4) + padded(mcap * 16) + 2 * padded(4);
    st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    SpmvArgs a;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.val = val;
    a.x = x;
    a.y = y;
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.chunk = chunk;
    a.big = cfg.block * cfg.items_per_lane;
    a.chunks = pool_take<int4>(ctx, cap);
    a.chunk_cap = cap;
    a.partials = pool_take<float>(ctx, cap);
    a.multi = pool_take<int4>(ctx, mcap);
    a.chunk_tail = pool_take<int>(ctx, 1);
    a.multi_tail = pool_take<int>(ctx, 1);
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;

    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    const int grid = (int)std::max<long long>(1, std::min<long long>(cfg.grid, (n + cfg.block - 1) / cfg.block));
    void *args[] = {&a};
    static const char *parent_names[] = {"spmv_parent_flat", "spmv_parent_wave", "spmv_parent_block",
                                         "spmv_parent_grid"};
    if (mode == WC_GRID) {
        st = launch(ctx, "spmv_reset", reinterpret_cast<const void *>(&spmv_reset), dim3(1), dim3(64), args, stream);
        if (st != WC_OK) return st;
    }
    st = launch(ctx, parent_names[mode], ks.parent, dim3(grid), dim3(cfg.block), args, stream);
    if (st != WC_OK) return st;
    if (mode == WC_GRID) {
        const int dgrid = std::max(1, std::min(cfg.grid, resident));
        st = launch(ctx, "spmv_drain", ks.drain, dim3(dgrid), dim3(cfg.block), args, stream);
        if (st == WC_OK) st = launch(ctx, "spmv_combine", ks.combine, dim3(dgrid), dim3(cfg.block), args, stream);
        if (st != WC_OK) return st;
    }
    return end_call(ctx, stream, stats, 1, cfg.fail_on_overflow);
}
