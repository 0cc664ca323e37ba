// SpMV with workload consolidation (irregular loop over CSR rows).
//
// One parent work item per row.  Prework reads the row's range; a row with
// more than `threshold` nonzeros is inserted into the consolidation buffer of
// its mode, a lighter row is summed inline by its lane ("work").
//   wave  - ballot-mask buffer; the wave sums its buffered rows.
//   block - LDS buffer, then the workgroup barrier; the block's waves sum the
//           buffered rows.
//   In both, the child sizes its lanes per row as grid mode does (below): g =
//   the power of two >= len / items_per_lane lanes per row, lane l of a group
//   taking elements l, l+g, ..., then a fixed butterfly over the group; the
//   rows of one g go 64 / g to a wave step.  A buffered row too long for one
//   group's child (more than one
//   chunk, 64 * items_per_lane nonzeros) is handed on as chunks to a global
//   buffer that the grid-mode drain spreads over the whole grid after the
//   parent (the KC_X rule of Sec. IV.E gives a warp's or block's child many
//   blocks); its chunk partials are combined in chunk order.
//   grid  - global buffers and a grid-wide barrier (kernel boundary).  The
//           child-work thread-count heuristic sizes the group of lanes that
//           sums one buffered row: g = the power of two >= len / items_per_lane,
//           so each lane takes about items_per_lane nonzeros.  Rows are binned by
//           g (1..64) and one wave sums 64 / g rows of a bin at once; a row
//           longer than 64 * items_per_lane is split into chunks of that size,
//           one wave each, and its chunk partials are combined in chunk order.
//           A counting pass sizes the bins before the parent pass fills them.
//   flat  - every row is summed by its own lane.
// All sums are fp32 fused multiply-adds whose order depends only on the row
// length, the mode and the tune, so results are bitwise reproducible.  Every
// serial part of a sum (a lane's share of a row, a wave's chunk partials) goes
// through a Cascade, so no product is rounded more than ~140 times on the way
// to y for rows of up to 2^26 nonzeros in any mode; 140 * 2^-24 < 1e-5, so
// |y - y_ref| <= 1e-5 * sum |a_ij x_j| holds as a worst-case bound per row.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

constexpr int kBins = 7;      // group sizes 1, 2, 4, ..., 64 lanes
constexpr int kChunkBin = 7;  // rows split into whole-wave chunks
constexpr int kUnroll = 4;    // nonzeros in flight per lane
constexpr int kMultiCol = 8;  // column of the per-block counts holding split rows
constexpr int kCols = 9;

struct SpmvArgs {
    const int *row_ptr;
    const int *col;
    const float *val;  // nullptr: every stored entry is 1 (the in-edge sums of PageRank)
    const float *x;
    float *y;
    // hot-column layout (wc_spmv_hot): column c < hot is the c-th most used
    // column, whose x value is x_hot[c]; column hot + j is column j of x
    const float *x_hot;
    const int *hot_ids;
    int hot;
    int n;
    int threshold;
    int ipl;           // items per lane
    int chunk;         // 64 * ipl
    int spill;         // wave and block modes: buffered rows longer than this go to the global chunks
    int count_drain;   // grid mode: the drain counts as the consolidated dispatch
    // grid mode
    int *blk_count;    // [grid * kCols]: per parent block, rows per bin 0..6, chunks, split rows
    int *blk_off;      // [grid * kCols]: exclusive offsets of each block within its column
    int *bin_total;    // [kCols]: column totals
    int4 *rows_buf;    // binned rows: (row, begin, end, 0), bins laid out by prefix of totals
    long long rows_cap;
    int4 *chunks;      // (row, begin, end, 0)
    long long chunk_cap;
    int4 *multi;       // (row, first chunk, chunk count, 0)
    long long multi_cap;
    float *partials;   // one per chunk slot
    DevStats *stats;
    int want_stats;
};

// x value of stored column c.  Plain layout (hot = 0): x[c].  Hot-column
// layout: the first nlds hot values staged in LDS (xs), the other hot ones in
// x_hot, the rest in x.
__device__ __forceinline__ float load_x(const SpmvArgs &a, const float *xs, int nlds, int c)
{
    if (c < a.hot) return c < nlds ? xs[c] : a.x_hot[c];
    return a.x[c - a.hot];
}

// Sum of val[e] * x[col[e]] over e = first + k * stride (k >= 0, e < end), in
// order of k, U loads in flight; the U products of a step are fused into the
// cascade's first partial sum one after another.
template <int U>
__device__ __forceinline__ float dot_strided_u(const SpmvArgs &a, int first, int stride, int end,
                                               const float *xs = nullptr, int nlds = 0)
{
    Cascade cs;
    for (int e0 = first; e0 < end; e0 += U * stride) {
        int c[U];
        float v[U], xv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int e = e0 + k * stride;
            const bool ok = e < end;
            c[k] = ok ? a.col[e] : -1;
            v[k] = ok ? (a.val ? a.val[e] : 1.f) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) xv[k] = c[k] >= 0 ? load_x(a, xs, nlds, c[k]) : 0.f;
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (c[k] >= 0) cs.s0 = fmaf(v[k], xv[k], cs.s0);
        cs.step<U>();
    }
    return cs.total();
}

__device__ __forceinline__ float dot_strided(const SpmvArgs &a, int first, int stride, int end)
{
    return dot_strided_u<kUnroll>(a, first, stride, end);
}

__device__ __forceinline__ float dot_wave(const SpmvArgs &a, int beg, int end)
{
    return wave_sum(dot_strided(a, beg + lane_id(), kWave, end));
}

// Sum over aligned groups of g lanes (g a power of two <= 64), fixed order.
__device__ __forceinline__ float group_sum(float v, int g)
{
    for (int d = g >> 1; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ int bin_of(int len, int ipl)
{
    // g = smallest power of two with g * ipl >= len, as a bin index (log2 g)
    int need = (len + ipl - 1) / ipl;
    int b = 0;
    while ((1 << b) < need) ++b;
    return b;
}

template <int BLOCK>
struct SpmvBlockBuf {
    int row[BLOCK];  // buffered rows, laid out by bin
    int beg[BLOCK];
    int end[BLOCK];
    int cnt[kBins + 1];   // rows per bin; [kBins]: heavy rows (work counters)
    int off[kBins];       // first row of each bin
    int task[kBins + 1];  // first task of each bin; [kBins]: task count
};

__device__ __forceinline__ void count_stats(StatAcc &acc, int len, bool heavy, bool wave_dispatch)
{
    acc.edges += len;
    acc.buffered += heavy ? len : 0;
    acc.items += heavy ? 1 : 0;
    if (wave_dispatch && __ballot(heavy) && lane_id() == 0) acc.dispatches += 1;
}

// Hands the rows of the lanes with nch > 0 on as chunks of the global buffer
// (wave and block modes): one reservation per wave for the chunks and one for
// the split-row records; the wave writes each row's chunks together.  A row
// whose chunks do not all fit is summed by its own lane instead (the overflow
// fallback) and its reserved entries are marked empty.  Every lane calls this.
__device__ __forceinline__ void spill_rows(const SpmvArgs &a, int r, int beg, int end, int nch)
{
    const int slot = wave_reserve_n(nch, &a.bin_total[kChunkBin]);
    const int mslot = wave_reserve(nch > 0, &a.bin_total[kMultiCol]);
    const bool fits = nch > 0 && (long long)slot + nch <= a.chunk_cap && mslot < a.multi_cap;
    uint64_t m = __ballot(fits);
    while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int s0 = readlane(slot, b), n0 = readlane(nch, b), rb = readlane(beg, b), re = readlane(end, b);
        const int rr = readlane(r, b);
        for (int c = lane_id(); c < n0; c += kWave) {
            const int cb = rb + c * a.chunk;
            a.chunks[s0 + c] = make_int4(rr, cb, min(re, cb + a.chunk), 0);
        }
    }
    if (fits) a.multi[mslot] = make_int4(r, slot, nch, 0);
    if (nch > 0 && !fits) {
        for (int c = 0; c < nch; ++c)
            if ((long long)slot + c < a.chunk_cap) a.chunks[slot + c] = make_int4(-1, 0, 0, 0);
        if (mslot < a.multi_cap) a.multi[mslot] = make_int4(-1, 0, 0, 0);
        a.stats->overflowed = 1;
        a.y[r] = dot_strided(a, beg, 1, end);
    }
}

// Zeroes the bin totals before a wave- or block-mode parent reserves chunks.
__global__ void spmv_reset(SpmvArgs a)
{
    if (threadIdx.x < kCols) a.bin_total[threadIdx.x] = 0;
}

// Parent kernel of the flat, wave and block modes.
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_parent(SpmvArgs a)
{
    const int lane = lane_id();
    StatAcc acc;
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
        if (a.want_stats) count_stats(acc, len, heavy, MODE == WC_WAVE);
        if (valid && !heavy) a.y[r] = dot_strided(a, beg, 1, end);
        // buffered rows too long for the group's own child go to the global chunks
        const bool spill = heavy && len > a.spill;
        if constexpr (MODE != WC_FLAT) {
            if (__ballot(spill)) spill_rows(a, r, beg, end, spill ? (len + a.chunk - 1) / a.chunk : 0);
        }
        const bool mine = heavy && !spill;

        // the child: the scope's buffered rows grouped by bin, g = 2^b lanes
        // per row (the smallest group that covers the row at items_per_lane
        // nonzeros a lane), 64 / g rows a wave step
        const int bin = mine ? bin_of(len, a.ipl) : -1;
        if constexpr (MODE == WC_WAVE) {
            const int wbase = base + (threadIdx.x & ~(kWave - 1));
            for (int b = 0; b < kBins; ++b) {
                const uint64_t m = __ballot(bin == b);
                if (!m) continue;
                // lane k learns which lane holds the bin's k-th row: the
                // members go to slots 0..cnt-1, the others after them, so the
                // permutation writes every lane once
                const int cnt = __popcll(m);
                const int to = bin == b ? rank_in(m) : cnt + rank_in(~m);
                const int src = __builtin_amdgcn_ds_permute(to << 2, lane);
                const int g = 1 << b, sub = lane & (g - 1);
                for (int i0 = 0; i0 < cnt; i0 += kWave >> b) {
                    const int i = i0 + (lane >> b);
                    const int from = __shfl(src, i < cnt ? i : 0, kWave);
                    const int rb = __shfl(beg, from, kWave), re = __shfl(end, from, kWave);
                    float s = dot_strided(a, i < cnt ? rb + sub : 0, g, i < cnt ? re : 0);
                    s = group_sum(s, g);
                    if (i < cnt && sub == 0) a.y[wbase + from] = s;
                }
            }
        } else if constexpr (MODE == WC_BLOCK) {
            __shared__ SpmvBlockBuf<BLOCK> sb;
            constexpr int NW = BLOCK / kWave;
            // per-bin insert positions: a row's sum depends only on its own
            // range and g, not on where it sits, so LDS atomics may order a bin
            if (threadIdx.x <= kBins) sb.cnt[threadIdx.x] = 0;
            __syncthreads();
            const int k = bin >= 0 ? atomicAdd(&sb.cnt[bin], 1) : 0;
            if (a.want_stats && heavy) atomicAdd(&sb.cnt[kBins], 1);
            __syncthreads();
            if (threadIdx.x == 0) {
                int o = 0, t = 0;
                for (int b = 0; b < kBins; ++b) {
                    sb.off[b] = o;
                    sb.task[b] = t;
                    o += sb.cnt[b];
                    t += (sb.cnt[b] + (kWave >> b) - 1) / (kWave >> b);
                }
                sb.task[kBins] = t;
                if (a.want_stats && sb.cnt[kBins]) acc.dispatches += 1;
            }
            __syncthreads();
            if (bin >= 0) {
                const int q = sb.off[bin] + k;
                sb.row[q] = r;
                sb.beg[q] = beg;
                sb.end[q] = end;
            }
            __syncthreads();  // the "synchronize" between inserts and the child
            // tasks of 64 / g rows of one bin, dealt round-robin to the waves
            const int total = sb.task[kBins];
            for (int t = threadIdx.x / kWave; t < total; t += NW) {
                int b = 0;
                while (b + 1 < kBins && sb.task[b + 1] <= t) ++b;
                const int g = 1 << b, sub = lane & (g - 1);
                const int i = (t - sb.task[b]) * (kWave >> b) + (lane >> b);
                const bool ok = i < sb.cnt[b];
                const int q = sb.off[b] + (ok ? i : 0);
                float s = dot_strided(a, ok ? sb.beg[q] + sub : 0, g, ok ? sb.end[q] : 0);
                s = group_sum(s, g);
                if (ok && sub == 0) a.y[sb.row[q]] = s;
            }
            __syncthreads();  // LDS buffer is reused by the next window
        }
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// ---- grid mode --------------------------------------------------------------------------------

// Counting pass: each parent block counts, over exactly the rows it will take
// in the parent pass, its rows per bin, its chunks of split rows and its split
// rows.  No atomics: one row of counts per block.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_classify(SpmvArgs a)
{
    __shared__ int cnt[kCols];
    if (threadIdx.x < kCols) cnt[threadIdx.x] = 0;
    __syncthreads();
    int mine[kCols];
#pragma unroll
    for (int c = 0; c < kCols; ++c) mine[c] = 0;
    // four windows' row lengths are requested together
    constexpr int W = 4;
    const int stride = gridDim.x * BLOCK;
    for (long long base0 = (long long)blockIdx.x * BLOCK; base0 < a.n; base0 += (long long)W * stride) {
        int lens[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const long long r = base0 + (long long)w * stride + threadIdx.x;
            lens[w] = r < a.n ? a.row_ptr[r + 1] - a.row_ptr[r] : 0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int len = lens[w];
            if (len > a.threshold) {
                if (len > a.chunk) {
                    mine[kChunkBin] += (len + a.chunk - 1) / a.chunk;
                    mine[kMultiCol] += 1;
                } else {
                    const int b = bin_of(len, a.ipl);
#pragma unroll
                    for (int c = 0; c < kBins; ++c) mine[c] += c == b;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kCols; ++c) {
        int v = wave_sum_i(mine[c]);
        if (lane_id() == 0 && v) atomicAdd(&cnt[c], v);
    }
    __syncthreads();
    if (threadIdx.x < kCols) a.blk_count[blockIdx.x * kCols + threadIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of the per-block counts down each column: one workgroup, one
// wave per column; a wave requests 16 x 64 counts at once, then scans them
// with wave scans and a running carry (no barriers).
__global__ __launch_bounds__(kCols * kWave) void spmv_scan(SpmvArgs a, int nblocks)
{
    constexpr int K = 16;
    const int c = threadIdx.x / kWave, lane = lane_id();
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += K * kWave) {
        int v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int b = b0 + k * kWave + lane;
            v[k] = b < nblocks ? a.blk_count[b * kCols + c] : 0;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int b = b0 + k * kWave + lane;
            const int incl = wave_incl_scan(v[k]);
            if (b < nblocks) a.blk_off[b * kCols + c] = carry + incl - v[k];
            carry += __shfl(incl, kWave - 1, kWave);
        }
    }
    if (lane == 0) a.bin_total[c] = carry;
}

// Parent pass of grid mode: light rows inline, heavy rows written into their
// bin at the offsets the scan gave this block.  STATS: the instantiation that
// counts work for wc_stats (without it no counters are kept live).
template <int BLOCK, bool STATS>
__global__ __launch_bounds__(BLOCK) void spmv_parent_grid(SpmvArgs a)
{
    __shared__ int cur[kCols], binoff[kBins], cnt[kCols];
    StatAcc acc;
    if (threadIdx.x < kCols) cur[threadIdx.x] = a.blk_off[blockIdx.x * kCols + threadIdx.x];
    if (threadIdx.x == 0) {
        int o = 0;
        for (int b = 0; b < kBins; ++b) {
            binoff[b] = o;
            o += a.bin_total[b];
        }
    }
    for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {
        if (threadIdx.x < kCols) cnt[threadIdx.x] = 0;
        __syncthreads();
        const int r = base + threadIdx.x;
        const bool valid = r < a.n;
        int beg = 0, end = 0;
        if (valid) {
            beg = a.row_ptr[r];
            end = a.row_ptr[r + 1];
        }
        const int len = end - beg;
        const bool heavy = len > a.threshold;
        if (STATS) count_stats(acc, len, heavy, false);
        if (valid && !heavy) a.y[r] = dot_strided_u<2 * kUnroll>(a, beg, 1, end);
        int bin = -1, local = 0, nch = 0, mlocal = 0;
        if (heavy) {
            if (len > a.chunk) {
                bin = kChunkBin;
                nch = (len + a.chunk - 1) / a.chunk;
                local = atomicAdd(&cnt[kChunkBin], nch);
                mlocal = atomicAdd(&cnt[kMultiCol], 1);
            } else {
                bin = bin_of(len, a.ipl);
                local = atomicAdd(&cnt[bin], 1);
            }
        }
        __syncthreads();
        if (bin >= 0 && bin < kBins) {
            const long long pos = (long long)binoff[bin] + cur[bin] + local;
            if (pos < a.rows_cap) a.rows_buf[pos] = make_int4(r, beg, end, 0);
        }
        // split rows: the wave writes each such row's chunks together (a long
        // row's chunks are not left to its own lane)
        const int slot = cur[kChunkBin] + local;
        const bool split_fits = bin == kChunkBin && (long long)slot + nch <= a.chunk_cap;
        uint64_t cm = __ballot(split_fits);
        while (cm) {
            const int b = __builtin_ctzll(cm);
            cm &= cm - 1;
            const int s0 = readlane(slot, b), n0 = readlane(nch, b);
            const int rb = readlane(beg, b), re = readlane(end, b), rr = readlane(r, b);
            for (int c = lane_id(); c < n0; c += kWave) {
                const int cb = rb + c * a.chunk;
                a.chunks[s0 + c] = make_int4(rr, cb, min(re, cb + a.chunk), 0);
            }
        }
        if (bin == kChunkBin) {
            const long long mpos = (long long)cur[kMultiCol] + mlocal;
            if (split_fits) {
                if (mpos < a.multi_cap) a.multi[mpos] = make_int4(r, slot, nch, 0);
            } else {
                // buffer full: mark the reserved slots that exist as empty and
                // sum the row inline (fallback); its split-row entry combines nothing
                for (int c = 0; c < nch; ++c)
                    if ((long long)slot + c < a.chunk_cap) a.chunks[slot + c] = make_int4(-1, 0, 0, 0);
                a.stats->overflowed = 1;
                a.y[r] = dot_strided(a, beg, 1, end);
                if (mpos < a.multi_cap) a.multi[mpos] = make_int4(-1, 0, 0, 0);
            }
        }
        __syncthreads();
        if (threadIdx.x < kCols) cur[threadIdx.x] += cnt[threadIdx.x];
    }
    if (STATS) stat_flush(a.stats, acc);
}

// Grid mode with the buffers of an earlier product on the same matrix still in
// place (PageRank's later sweeps): only the rows up to the threshold, summed
// inline as spmv_parent_grid sums them; the binned rows and chunks are reused.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_light_rows(SpmvArgs a)
{
    for (int r = blockIdx.x * BLOCK + threadIdx.x; r < a.n; r += gridDim.x * BLOCK) {
        const int beg = a.row_ptr[r], end = a.row_ptr[r + 1];
        if (end - beg <= a.threshold) a.y[r] = dot_strided_u<2 * kUnroll>(a, beg, 1, end);
    }
}

// Consolidated child of grid mode.  Wave tasks: for bin b (g = 2^b lanes per
// row) a task is 64 / g consecutive rows of the bin; then one task per chunk.
// Hot x values staged in LDS by the drain of the hot-column layout: 32 per
// thread, at most 16384 (64 KiB), so that four waves per SIMD stay resident.
template <int BLOCK>
constexpr int lds_hot_for() { return 32 * BLOCK < 16384 ? 32 * BLOCK : 16384; }

template <int BLOCK, bool HOT>
struct DrainLds {
    float x[HOT ? lds_hot_for<BLOCK>() : 1];
};

template <int BLOCK, bool HOT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(HOT ? 4 : 8))) void spmv_drain(SpmvArgs a)
{
    __shared__ int s_cnt[8], s_off[8], s_task[9];
    __shared__ DrainLds<BLOCK, HOT> s_x;
    const int nlds = HOT ? min(a.hot, lds_hot_for<BLOCK>()) : 0;
    if (HOT)
        for (int i = threadIdx.x; i < nlds; i += BLOCK) s_x.x[i] = a.x_hot[i];
    if (threadIdx.x == 0) {
        int o = 0, t = 0;
        for (int b = 0; b < 8; ++b) {
            int c = a.bin_total[b];
            if (b == kChunkBin) c = (long long)c < a.chunk_cap ? c : (int)a.chunk_cap;
            s_cnt[b] = c;
            s_off[b] = o;
            if (b < kBins) o += c;
            s_task[b] = t;
            t += b < kBins ? (c + (kWave >> b) - 1) / (kWave >> b) : c;
        }
        s_task[8] = t;
        if (a.want_stats && a.count_drain && blockIdx.x == 0 && t > 0)
            atomic_add_dev(&a.stats->rep[0].dispatches, 1ull);
    }
    __syncthreads();
    const int total = s_task[8];
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    const int lane = lane_id();
    for (int t = gw; t < total; t += nw) {
        int b = 0;
        while (b < 7 && s_task[b + 1] <= t) ++b;
        // bin task: groups of g lanes per row; chunk task: the whole wave on
        // one chunk (g = 64).  One code path, so one copy of the dot product.
        const bool chunk = b >= kBins;
        const int g = chunk ? kWave : 1 << b;
        const int sub = lane & (g - 1);
        int first = 0, end = 0, dst = -1;
        if (chunk) {
            const int c = t - s_task[kChunkBin];
            const int4 d = a.chunks[c];
            if (__builtin_amdgcn_readfirstlane(d.x) >= 0) {
                first = __builtin_amdgcn_readfirstlane(d.y) + lane;
                end = __builtin_amdgcn_readfirstlane(d.z);
                dst = c;
            }
        } else {
            const int i = (t - s_task[b]) * (kWave >> b) + (lane >> b);
            if (i < s_cnt[b]) {
                const int4 d = a.rows_buf[s_off[b] + i];
                first = d.y + sub;
                end = d.z;
                dst = d.x;
            }
        }
        float s = dot_strided_u<2 * kUnroll>(a, first, g, end, s_x.x, nlds);
        s = group_sum(s, g);
        if (dst >= 0 && sub == 0) {
            if (chunk) a.partials[dst] = s;
            else a.y[dst] = s;
        }
    }
}

// Post-work of split rows: the chunk partials of each row, summed in chunk order.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_combine(SpmvArgs a)
{
    const int total = (int)min((long long)a.bin_total[kMultiCol], a.multi_cap);
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    for (int i = gw; i < total; i += nw) {
        int4 d = a.multi[i];
        const int row = __builtin_amdgcn_readfirstlane(d.x);
        if (row < 0) continue;
        int first = __builtin_amdgcn_readfirstlane(d.y), cnt = __builtin_amdgcn_readfirstlane(d.z);
        Cascade cs;
        for (int c = lane_id(); c < cnt; c += kWave) cs.add(a.partials[first + c]);
        const float s = wave_sum(cs.total());
        if (lane_id() == 0) a.y[row] = s;
    }
}

// basic dynamic parallelism, emulated for comparison (driver 2): the parent
// sums the light rows inline and lists the heavy ones; the host then launches
// one child per listed row (no consolidation).
constexpr int kBasicBlock = 256;
__global__ __launch_bounds__(kBasicBlock) void spmv_parent_basic(SpmvArgs a)
{
    for (int base = blockIdx.x * kBasicBlock; base < a.n; base += gridDim.x * kBasicBlock) {
        const int r = base + threadIdx.x;
        const bool valid = r < a.n;
        int beg = 0, end = 0;
        if (valid) {
            beg = a.row_ptr[r];
            end = a.row_ptr[r + 1];
        }
        const bool heavy = valid && end - beg > a.threshold;
        if (valid && !heavy) a.y[r] = dot_strided(a, beg, 1, end);
        const int s = wave_reserve(heavy, &a.bin_total[0]);
        if (heavy && s < a.rows_cap) a.rows_buf[s] = make_int4(r, beg, end, 0);
    }
}

// The child of ONE heavy row: one workgroup strides over the row, then a
// fixed-order workgroup sum.
__global__ __launch_bounds__(kBasicBlock) void spmv_child_basic(SpmvArgs a, int r, int beg, int end)
{
    __shared__ float tmp[kBasicBlock / kWave];
    const float s = block_sum<kBasicBlock>(dot_strided(a, beg + (int)threadIdx.x, kBasicBlock, end), tmp);
    if (threadIdx.x == 0) a.y[r] = s;
}

__global__ void spmv_basic_reset(SpmvArgs a)
{
    if (threadIdx.x == 0) a.bin_total[0] = 0;
}

// x_hot[k] = x[hot_ids[k]] for the hot-column layout (once per product).
__global__ __launch_bounds__(256) void spmv_gather_hot(SpmvArgs a)
{
    float *xh = const_cast<float *>(a.x_hot);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < a.hot; k += gridDim.x * 256) xh[k] = a.x[a.hot_ids[k]];
}

struct SpmvKernels {
    const void *parent, *classify, *parent_grid, *drain, *combine, *light;
};

template <int BLOCK>
SpmvKernels pick_block(wc_mode mode, bool hot, bool stats)
{
    SpmvKernels k{nullptr, reinterpret_cast<const void *>(&spmv_classify<BLOCK>),
                  stats ? reinterpret_cast<const void *>(&spmv_parent_grid<BLOCK, true>)
                        : reinterpret_cast<const void *>(&spmv_parent_grid<BLOCK, false>),
                  hot ? reinterpret_cast<const void *>(&spmv_drain<BLOCK, true>)
                      : reinterpret_cast<const void *>(&spmv_drain<BLOCK, false>),
                  reinterpret_cast<const void *>(&spmv_combine<BLOCK>),
                  reinterpret_cast<const void *>(&spmv_light_rows<BLOCK>)};
    switch (mode) {
    case WC_FLAT: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_FLAT, BLOCK>); break;
    case WC_WAVE: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_WAVE, BLOCK>); break;
    case WC_BLOCK: k.parent = reinterpret_cast<const void *>(&spmv_parent<WC_BLOCK, BLOCK>); break;
    default: k.parent = k.parent_grid; break;
    }
    return k;
}

SpmvKernels pick(wc_mode mode, int block, bool hot, bool stats)
{
    switch (block) {
    case 64: return pick_block<64>(mode, hot, stats);
    case 128: return pick_block<128>(mode, hot, stats);
    case 512: return pick_block<512>(mode, hot, stats);
    case 1024: return pick_block<1024>(mode, hot, stats);
    default: return pick_block<256>(mode, hot, stats);
    }
}


// A planned product y = A x: the tune resolved, the kernels picked and the
// workspace laid out (plus `extra_bytes` left for the caller after it).  x and
// y may be set after planning.
struct SpmvPlan {
    SpmvArgs a;
    SpmvKernels ks;
    Config cfg;
    wc_mode mode;
    int grid, dgrid;
    long long rows_cap, cap, mcap;
};

// Resolves the tune and the launch shapes for a device with `num_cus` compute
// units; touches no memory.
wc_status spmv_shape(int num_cus, const wc_csr *g, const float *val, wc_mode mode, const wc_tune *tune,
                     bool want_stats, SpmvPlan *p, bool hot = false)
{
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    p->mode = mode;
    p->ks = pick(mode, block, hot, want_stats);
    int resident = resident_blocks_on(num_cus, p->ks.parent, block);
    wc_status st = resolve_tune(nullptr, "spmv", mode, tune, resident, &p->cfg);
    if (st != WC_OK) return st;
    const Config &cfg = p->cfg;
    if (cfg.block != block) {
        p->ks = pick(mode, cfg.block, hot, want_stats);
        resident = resident_blocks_on(num_cus, p->ks.parent, cfg.block);
    }
    // the drain of the hot-column layout holds 64 KiB of LDS: its own residency
    if (hot) resident = std::min(resident, resident_blocks_on(num_cus, p->ks.drain, cfg.block));
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    // wave and block modes hand rows longer than `spill` (one chunk) on as
    // chunks: at most m / spill such rows, each with at most one partly filled chunk
    const int spill = chunk;
    long long cap_full = n + m / chunk + 1, multi_full = n;
    if (mode == WC_WAVE || mode == WC_BLOCK) {
        cap_full = m / chunk + m / spill + 1;
        multi_full = m / spill + 1;
    }
    p->cap = mode != WC_FLAT ? (cfg.buf_capacity > 0 ? std::min(cfg.buf_capacity, cap_full) : cap_full) : 1;
    p->rows_cap = mode == WC_GRID ? n : 1;
    p->mcap = mode != WC_FLAT ? multi_full : 1;
    // wave and block modes launch the parent with a thread per row (one window
    // per workgroup) unless grid_blocks caps it: the hardware hands windows to
    // CUs as they free up, which evens out the windows dense with buffered rows
    // (scale-22 graph: wave 0.92 -> 0.85 ms, block 0.93 -> 0.85 ms against the
    // resident grid)
    const long long windows = (n + cfg.block - 1) / cfg.block;
    const bool own_grid = tune && tune->grid_blocks > 0;
    p->grid = (int)std::max<long long>(1, (mode == WC_WAVE || mode == WC_BLOCK) && !own_grid
                                              ? windows
                                              : std::min<long long>(cfg.grid, windows));
    p->dgrid = std::max(1, std::min(cfg.grid, resident));
    SpmvArgs &a = p->a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.val = val;
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.ipl = cfg.items_per_lane;
    a.chunk = chunk;
    a.spill = spill;
    a.count_drain = mode == WC_GRID;
    a.rows_cap = p->rows_cap;
    a.chunk_cap = p->cap;
    a.multi_cap = p->mcap;
    a.want_stats = want_stats;
    return WC_OK;
}

// Rows of the per-parent-block counts and offsets: grid mode's count pass
// only.
size_t blk_rows(const SpmvPlan *p) { return p->mode == WC_GRID ? (size_t)p->grid : 1; }

// Bytes of workspace the planned product needs (256-byte aligned pieces).
size_t spmv_workspace_bytes(const SpmvPlan *p)
{
    return 2 * padded(blk_rows(p) * kCols * 4) + padded(kCols * 4) + padded(p->rows_cap * 16) + padded(p->cap * 16) +
           padded(p->cap * 4) + padded(p->mcap * 16);
}

// Lays the workspace out from `base` (256-byte aligned, spmv_workspace_bytes
// long); returns the first byte after it.
char *spmv_carve(SpmvPlan *p, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = base + off;
        off += padded(bytes);
        return q;
    };
    SpmvArgs &a = p->a;
    a.blk_count = reinterpret_cast<int *>(take(blk_rows(p) * kCols * 4));
    a.blk_off = reinterpret_cast<int *>(take(blk_rows(p) * kCols * 4));
    a.bin_total = reinterpret_cast<int *>(take(kCols * 4));
    a.rows_buf = reinterpret_cast<int4 *>(take(p->rows_cap * 16));
    a.chunks = reinterpret_cast<int4 *>(take(p->cap * 16));
    a.partials = reinterpret_cast<float *>(take(p->cap * 4));
    a.multi = reinterpret_cast<int4 *>(take(p->mcap * 16));
    return base + off;
}

wc_status spmv_plan(wc_ctx *ctx, const wc_csr *g, const float *val, wc_mode mode, const wc_tune *tune,
                    size_t extra_bytes, hipStream_t stream, wc_stats *stats, SpmvPlan *p, bool hot = false)
{
    wc_status st = spmv_shape(ctx->num_cus, g, val, mode, tune, stats != nullptr, p, hot);
    if (st != WC_OK) return st;
    st = pool_reserve(ctx, spmv_workspace_bytes(p) + extra_bytes, stream);
    if (st != WC_OK) return st;
    char *end = spmv_carve(p, ctx->pool);
    ctx->pool_off = (size_t)(end - ctx->pool);
    p->a.stats = ctx->dstats;
    return WC_OK;
}

// The kernels of one product (parent; in grid mode classify, scan, parent,
// drain, combine).
wc_status spmv_launch(wc_ctx *ctx, SpmvPlan *p, hipStream_t stream)
{
    const Config &cfg = p->cfg;
    void *args[] = {&p->a};
    if (p->mode == WC_FLAT)
        return launch(ctx, "spmv_parent_flat", p->ks.parent, dim3(p->grid), dim3(cfg.block), args, stream);
    if (p->mode != WC_GRID) {
        // parent, then the grid-wide drain of the rows it handed on and their combination
        const char *name = p->mode == WC_WAVE ? "spmv_parent_wave" : "spmv_parent_block";
        wc_status st = launch(ctx, "spmv_reset", reinterpret_cast<const void *>(&spmv_reset), dim3(1), dim3(kWave),
                              args, stream);
        if (st == WC_OK) st = launch(ctx, name, p->ks.parent, dim3(p->grid), dim3(cfg.block), args, stream);
        if (st == WC_OK) st = launch(ctx, "spmv_drain", p->ks.drain, dim3(p->dgrid), dim3(cfg.block), args, stream);
        if (st == WC_OK)
            st = launch(ctx, "spmv_combine", p->ks.combine, dim3(p->dgrid), dim3(cfg.block), args, stream);
        return st;
    }
    int nblocks = p->grid;
    void *sargs[] = {&p->a, &nblocks};
    wc_status st = launch(ctx, "spmv_classify", p->ks.classify, dim3(p->grid), dim3(cfg.block), args, stream);
    if (st == WC_OK)
        st = launch(ctx, "spmv_scan", reinterpret_cast<const void *>(&spmv_scan), dim3(1), dim3(kCols * kWave), sargs,
                    stream);
    if (st == WC_OK)
        st = launch(ctx, "spmv_parent_grid", p->ks.parent_grid, dim3(p->grid), dim3(cfg.block), args, stream);
    if (st == WC_OK) st = launch(ctx, "spmv_drain", p->ks.drain, dim3(p->dgrid), dim3(cfg.block), args, stream);
    if (st == WC_OK) st = launch(ctx, "spmv_combine", p->ks.combine, dim3(p->dgrid), dim3(cfg.block), args, stream);
    return st;
}

// Grid mode, again on the same matrix with the buffers of the last spmv_launch
// of this plan still in place (full-size buffers, so nothing overflowed): the
// rows up to the threshold inline, then the drain and the combination of the
// reused binned rows and chunks.  Same sums, in the same order, as spmv_launch.
wc_status spmv_relaunch(wc_ctx *ctx, SpmvPlan *p, hipStream_t stream)
{
    const Config &cfg = p->cfg;
    void *args[] = {&p->a};
    wc_status st = launch(ctx, "spmv_light_rows", p->ks.light, dim3(p->grid), dim3(cfg.block), args, stream);
    if (st == WC_OK) st = launch(ctx, "spmv_drain", p->ks.drain, dim3(p->dgrid), dim3(cfg.block), args, stream);
    if (st == WC_OK) st = launch(ctx, "spmv_combine", p->ks.combine, dim3(p->dgrid), dim3(cfg.block), args, stream);
    return st;
}

// ---------------------------------------------------------------- PageRank

struct PrArgs {
    const int *out_degree;
    float *rank;
    float *contrib;   // rank[u] / outdeg(u), the x of the in-edge sums
    const float *sums;  // sum over the in-edges of v of contrib[u]
    float *dpart;     // per block of pr_contrib: rank held by vertices without out-edges
    int nparts;
    int n;
    float base;       // (1 - d) / n
    float damping;
    float inv_n;
};

constexpr int kPrBlock = 256;

__global__ __launch_bounds__(kPrBlock) void pr_init(PrArgs p)
{
    for (int v = blockIdx.x * kPrBlock + threadIdx.x; v < p.n; v += gridDim.x * kPrBlock) p.rank[v] = p.inv_n;
}

// contrib[u] = rank[u] / outdeg(u); the ranks of vertices without out-edges
// are summed per block in a fixed order into dpart[blockIdx.x].
__global__ __launch_bounds__(kPrBlock) void pr_contrib(PrArgs p)
{
    __shared__ float red[kPrBlock / kWave];
    Cascade dang;
    for (int u = blockIdx.x * kPrBlock + threadIdx.x; u < p.n; u += gridDim.x * kPrBlock) {
        const float r = p.rank[u];
        const int od = p.out_degree[u];
        p.contrib[u] = od > 0 ? r / (float)od : 0.f;
        dang.add(od == 0 ? r : 0.f);
    }
    const float dsum_block = block_sum<kPrBlock>(dang.total(), red);
    if (threadIdx.x == 0) p.dpart[blockIdx.x] = dsum_block;
}

// rank'[v] = (1 - d) / n + d * (sums[v] + D / n), D the sum of dpart in block
// order (every block computes the same D).
__global__ __launch_bounds__(kPrBlock) void pr_update(PrArgs p)
{
    __shared__ float red[kPrBlock / kWave];
    Cascade part;
    for (int i = threadIdx.x; i < p.nparts; i += kPrBlock) part.add(p.dpart[i]);
    const float dsum = block_sum<kPrBlock>(part.total(), red);
    const float spread = dsum * p.inv_n;
    for (int v = blockIdx.x * kPrBlock + threadIdx.x; v < p.n; v += gridDim.x * kPrBlock)
        p.rank[v] = p.base + p.damping * (p.sums[v] + spread);
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
    SpmvPlan p;
    wc_status st = spmv_plan(ctx, g, val, mode, tune, 0, stream, stats, &p);
    if (st != WC_OK) return st;
    p.a.x = x;
    p.a.y = y;
    if (p.cfg.driver == 1 || p.cfg.driver == 3 || (p.cfg.driver == 2 && mode != WC_GRID))
        return fail(WC_EINVAL, "wc_spmv: driver 2 needs grid mode; drivers 1 and 3 do not apply");
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    if (p.cfg.driver == 2) {
        // Basic dynamic parallelism, emulated: the host reads the heavy rows back
        // and launches one child per row.
        void *args[] = {&p.a};
        st = launch(ctx, "spmv_basic_reset", reinterpret_cast<const void *>(&spmv_basic_reset), dim3(1), dim3(64),
                    args, stream);
        const int bgrid = (int)std::min<long long>((g->n + kBasicBlock - 1) / kBasicBlock, 4LL * ctx->num_cus);
        if (st == WC_OK)
            st = launch(ctx, "spmv_parent_basic", reinterpret_cast<const void *>(&spmv_parent_basic), dim3(bgrid),
                        dim3(kBasicBlock), args, stream);
        if (st != WC_OK) return st;
        int tail = 0;
        WC_HIP(hipMemcpyAsync(&tail, p.a.bin_total, sizeof(int), hipMemcpyDeviceToHost, stream));
        WC_HIP(hipStreamSynchronize(stream));
        const int count = (int)std::min<long long>(tail, p.a.rows_cap);
        std::vector<int4> rows((size_t)std::max(count, 1));
        if (count > 0) WC_HIP(hipMemcpy(rows.data(), p.a.rows_buf, sizeof(int4) * (size_t)count, hipMemcpyDeviceToHost));
        chain_break(ctx);
        for (int i = 0; i < count; ++i) {
            int r = rows[i].x, beg = rows[i].y, end = rows[i].z;
            void *cargs[] = {&p.a, &r, &beg, &end};
            st = launch(ctx, "spmv_child_basic", reinterpret_cast<const void *>(&spmv_child_basic), dim3(1),
                        dim3(kBasicBlock), cargs, stream);
            if (st != WC_OK) return st;
        }
        st = end_call(ctx, stream, stats, 1, p.cfg.fail_on_overflow);
        if (stats) {
            stats->items_buffered = count;
            stats->dispatches = count;
        }
        return st;
    }
    st = spmv_launch(ctx, &p, stream);
    if (st != WC_OK) return st;
    return end_call(ctx, stream, stats, 1, p.cfg.fail_on_overflow);
}

extern "C" wc_status wc_pagerank(wc_ctx *ctx, const wc_csr *in_graph, const int32_t *out_degree, int32_t iterations,
                                 float damping, float *rank, wc_mode mode, const wc_tune *tune, hipStream_t stream,
                                 wc_stats *stats)
{
    if (!ctx || !in_graph) return fail(WC_EINVAL, "wc_pagerank: NULL context or graph");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_pagerank: bad mode");
    if (in_graph->n < 0 || in_graph->m < 0 || iterations < 0) return fail(WC_EINVAL, "wc_pagerank: negative size");
    if (!(damping >= 0.f && damping <= 1.f)) return fail(WC_EINVAL, "wc_pagerank: damping outside [0, 1]");
    if (in_graph->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (!in_graph->row_ptr || !out_degree || !rank || (in_graph->m > 0 && !in_graph->col))
        return fail(WC_EINVAL, "wc_pagerank: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    const long long n = in_graph->n;
    const int pgrid = (int)std::min<long long>((n + kPrBlock - 1) / kPrBlock, 4 * (long long)ctx->num_cus);
    SpmvPlan p;
    wc_status st = spmv_plan(ctx, in_graph, nullptr, mode, tune, 2 * padded(n * 4) + padded((size_t)pgrid * 4), stream,
                             stats, &p);
    if (st != WC_OK) return st;
    if (p.cfg.driver != 0) return fail(WC_EINVAL, "wc_pagerank: only the relaunch driver (driver = 0) applies");
    PrArgs q;
    q.out_degree = out_degree;
    q.rank = rank;
    q.contrib = pool_take<float>(ctx, n);
    float *sums = pool_take<float>(ctx, n);
    q.sums = sums;
    q.dpart = pool_take<float>(ctx, pgrid);
    q.nparts = pgrid;
    q.n = (int)n;
    q.base = (float)((1.0 - (double)damping) / (double)n);
    q.damping = damping;
    q.inv_n = (float)(1.0 / (double)n);
    p.a.x = q.contrib;
    p.a.y = sums;
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    void *args[] = {&q};
    st = launch(ctx, "pr_init", reinterpret_cast<const void *>(&pr_init), dim3(pgrid), dim3(kPrBlock), args, stream);
    // grid mode: the in-edge structure is the same every sweep, so the binned
    // rows and chunks of the first sweep serve the later ones (only when the
    // buffers are full size, so that nothing overflowed, and without work
    // counters, which count each sweep's binning)
    const bool reuse = mode == WC_GRID && !stats && !(tune && tune->buf_capacity > 0);
    for (int it = 0; it < iterations && st == WC_OK; ++it) {
        st = launch(ctx, "pr_contrib", reinterpret_cast<const void *>(&pr_contrib), dim3(pgrid), dim3(kPrBlock), args,
                    stream);
        if (st == WC_OK) st = reuse && it > 0 ? spmv_relaunch(ctx, &p, stream) : spmv_launch(ctx, &p, stream);
        if (st == WC_OK)
            st = launch(ctx, "pr_update", reinterpret_cast<const void *>(&pr_update), dim3(pgrid), dim3(kPrBlock),
                        args, stream);
    }
    if (st != WC_OK) return st;
    return end_call(ctx, stream, stats, iterations, p.cfg.fail_on_overflow);
}

// ---------------------------------------------------------------- hot-column layout

namespace wc {
namespace {

__global__ __launch_bounds__(256) void hot_count(const int *col, long long m, int *cnt)
{
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < m; e += (long long)gridDim.x * 256)
        atomicAdd(&cnt[col[e]], 1);
}

__global__ __launch_bounds__(256) void hot_remap(const int *col, long long m, const int *rank, int hot, int *out)
{
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < m; e += (long long)gridDim.x * 256) {
        const int c = col[e];
        const int r = rank[c];
        out[e] = r >= 0 ? r : hot + c;
    }
}

}  // namespace
}  // namespace wc

extern "C" wc_status wc_spmv_prepare(wc_ctx *ctx, const wc_csr *a, int32_t hot, int32_t *col_hot, int32_t *hot_ids,
                                     hipStream_t stream)
{
    if (!ctx || !a) return fail(WC_EINVAL, "wc_spmv_prepare: NULL context or matrix");
    if (a->n < 0 || a->m < 0) return fail(WC_EINVAL, "wc_spmv_prepare: negative size");
    if (hot < 0 || hot > a->n) return fail(WC_EINVAL, "wc_spmv_prepare: hot must be in [0, n]");
    if ((long long)a->n + hot > 0x7fffffffLL) return fail(WC_EINVAL, "wc_spmv_prepare: n + hot exceeds int32");
    if (a->n == 0) return WC_OK;
    if (!a->row_ptr || (a->m > 0 && (!a->col || !col_hot)) || (hot > 0 && !hot_ids))
        return fail(WC_EINVAL, "wc_spmv_prepare: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    const long long n = a->n, m = a->m;
    wc_status st = pool_reserve(ctx, 2 * padded(n * 4), stream);
    if (st != WC_OK) return st;
    int *cnt = pool_take<int>(ctx, n);
    int *rank = pool_take<int>(ctx, n);
    const int grid = (int)std::max<long long>(1, std::min<long long>((m + 255) / 256, 8LL * ctx->num_cus));
    chain_break(ctx);
    WC_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)n, stream));
    if (m > 0) {
        void *args[] = {const_cast<int **>(&a->col), const_cast<long long *>(&m), &cnt};
        st = launch(ctx, "hot_count", reinterpret_cast<const void *>(&hot_count), dim3(grid), dim3(256), args, stream);
        if (st != WC_OK) return st;
    }
    // the hot columns: most entries first, ties by column id
    std::vector<int> counts((size_t)n), order((size_t)n), rk((size_t)n, -1);
    WC_HIP(hipMemcpyAsync(counts.data(), cnt, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, stream));
    WC_HIP(hipStreamSynchronize(stream));
    for (long long v = 0; v < n; ++v) order[(size_t)v] = (int)v;
    auto more = [&](int u, int v) { return counts[u] != counts[v] ? counts[u] > counts[v] : u < v; };
    std::partial_sort(order.begin(), order.begin() + hot, order.end(), more);
    for (int k = 0; k < hot; ++k) rk[(size_t)order[(size_t)k]] = k;
    chain_break(ctx);
    WC_HIP(hipMemcpyAsync(rank, rk.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, stream));
    if (hot > 0) WC_HIP(hipMemcpyAsync(hot_ids, order.data(), sizeof(int) * (size_t)hot, hipMemcpyHostToDevice, stream));
    if (m > 0) {
        void *args[] = {const_cast<int **>(&a->col), const_cast<long long *>(&m), &rank, &hot, &col_hot};
        st = launch(ctx, "hot_remap", reinterpret_cast<const void *>(&hot_remap), dim3(grid), dim3(256), args, stream);
        if (st != WC_OK) return st;
    }
    // the host vectors above are read by the copies: wait for them
    WC_HIP(hipStreamSynchronize(stream));
    return WC_OK;
}

extern "C" wc_status wc_spmv_hot(wc_ctx *ctx, const wc_csr *a_hot, int32_t hot, const int32_t *hot_ids,
                                 const float *val, const float *x, float *y, wc_mode mode, const wc_tune *tune,
                                 hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !a_hot) return fail(WC_EINVAL, "wc_spmv_hot: NULL context or matrix");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_spmv_hot: bad mode");
    if (a_hot->n < 0 || a_hot->m < 0) return fail(WC_EINVAL, "wc_spmv_hot: negative size");
    if (hot < 0 || hot > a_hot->n) return fail(WC_EINVAL, "wc_spmv_hot: hot must be in [0, n]");
    if (a_hot->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (!a_hot->row_ptr || !x || !y || (a_hot->m > 0 && (!a_hot->col || !val)) || (hot > 0 && !hot_ids))
        return fail(WC_EINVAL, "wc_spmv_hot: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    SpmvPlan p;
    wc_status st = spmv_plan(ctx, a_hot, val, mode, tune, padded((size_t)std::max(hot, 1) * 4), stream, stats, &p,
                             hot > 0);
    if (st != WC_OK) return st;
    if (p.cfg.driver != 0) return fail(WC_EINVAL, "wc_spmv_hot: only the relaunch driver (driver = 0) applies");
    p.a.x = x;
    p.a.y = y;
    p.a.hot = hot;
    p.a.hot_ids = hot_ids;
    p.a.x_hot = pool_take<float>(ctx, (size_t)std::max(hot, 1));
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    if (hot > 0) {
        void *args[] = {&p.a};
        const int g = (int)std::min<long long>((hot + 255) / 256, 4LL * ctx->num_cus);
        st = launch(ctx, "spmv_gather_hot", reinterpret_cast<const void *>(&spmv_gather_hot), dim3(g), dim3(256), args,
                    stream);
        if (st != WC_OK) return st;
    }
    st = spmv_launch(ctx, &p, stream);
    if (st != WC_OK) return st;
    return end_call(ctx, stream, stats, 1, p.cfg.fail_on_overflow);
}

// ---------------------------------------------------------------- SpMV without allocation
//
// wc_spmv_noalloc: the kernels of wc_spmv with their workspace in a fixed
// device array instead of a context pool.  `scratch` is a host-side stand-in
// for that array: host code only ever uses the device address that
// hipGetSymbolAddress returns for it, taken once per device on the first call
// made with that device current.

static __device__ __align__(256) unsigned char scratch[WC_SPMV_NOALLOC_SCRATCH_BYTES];

namespace wc {
namespace {

constexpr int kMaxDevices = 64;
struct NoAllocDevice {
    bool ready = false;
    int num_cus = 0;
    char *scratch = nullptr;  // device address of `scratch` on this device
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kMaxDevices];

// Workspace bound from n, m and the tune alone (the parent grid at its
// largest, ceil(n / block)), so oversized calls are refused before any HIP
// call is made.
size_t spmv_noalloc_bound(const wc_csr *g, const SpmvPlan *p)
{
    SpmvPlan q = *p;
    q.grid = (int)std::max<long long>(1, ((long long)g->n + q.cfg.block - 1) / q.cfg.block);
    return spmv_workspace_bytes(&q) + padded(sizeof(DevStats));
}

}  // namespace
}  // namespace wc

extern "C" wc_status wc_spmv_noalloc(const wc_csr *g, const float *val, const float *x, float *y, wc_mode mode,
                                     const wc_tune *tune, hipStream_t stream)
{
    if (!g) return fail(WC_EINVAL, "wc_spmv_noalloc: NULL matrix");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_spmv_noalloc: bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, "wc_spmv_noalloc: negative size");
    if (g->n == 0) return WC_OK;
    if (!g->row_ptr || !x || !y || (g->m > 0 && (!g->col || !val)))
        return fail(WC_EINVAL, "wc_spmv_noalloc: NULL array");
    if (tune && tune->driver != 0)
        return fail(WC_EINVAL, "wc_spmv_noalloc: only the relaunch driver (driver = 0) applies");
    // the tune and the size limit are checked before any device memory is
    // touched; the compute-unit count only changes the drain grid, not the bound
    SpmvPlan p;
    wc_status st = spmv_shape(1, g, val, mode, tune, false, &p);
    if (st != WC_OK) return st;
    const size_t bound = spmv_noalloc_bound(g, &p);
    if (bound > (size_t)WC_SPMV_NOALLOC_SCRATCH_BYTES)
        return fail(WC_EINVAL, "wc_spmv_noalloc: the workspace (" + std::to_string(bound) +
                                   " bytes) exceeds the fixed scratch of " +
                                   std::to_string((size_t)WC_SPMV_NOALLOC_SCRATCH_BYTES) + " bytes");
    int dev = 0;
    WC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(WC_EINVAL, "wc_spmv_noalloc: device index out of range");
    NoAllocDevice d;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        NoAllocDevice &slot = g_noalloc[dev];
        if (!slot.ready) {
            int cus = 0;
            WC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            void *ptr = nullptr;
            WC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(WC_EHIP, "wc_spmv_noalloc: no device address for the scratch array");
            slot.num_cus = cus;
            slot.scratch = static_cast<char *>(ptr);
            slot.ready = true;
        }
        d = slot;
    }
    st = spmv_shape(d.num_cus, g, val, mode, tune, false, &p);
    if (st != WC_OK) return st;
    char *end = spmv_carve(&p, d.scratch);
    p.a.stats = reinterpret_cast<DevStats *>(end);  // written only on overflow, which a full-size buffer never has
    p.a.x = x;
    p.a.y = y;
    st = spmv_launch(nullptr, &p, stream);
    if (st != WC_OK) return st;
    WC_HIP(hipGetLastError());
    return WC_OK;
}
