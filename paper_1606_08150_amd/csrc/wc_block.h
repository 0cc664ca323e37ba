// Workgroup-level helpers: block-wide scans used to lay out LDS consolidation
// buffers in thread order (deterministic positions, no LDS atomics).
#pragma once

#include "wc_device.h"

namespace wc {

// Inclusive scan over the 64 lanes of a wave (all lanes active).
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int o = __shfl_up(v, d, kWave);
        v += lane >= d ? o : 0;
    }
    return v;
}

// Exclusive block scan of two ints at once.  `tmp` must hold 2 * (BLOCK/64) ints
// of LDS.  All threads of the block must call it.  Returns the exclusive
// prefixes and the block totals.
template <int BLOCK>
__device__ __forceinline__ void block_scan2(int a, int b, int *tmp, int &ea, int &eb, int &ta, int &tb)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int ia = wave_incl_scan(a), ib = wave_incl_scan(b);
    if (lane == kWave - 1) {
        tmp[wid] = ia;
        tmp[NW + wid] = ib;
    }
    __syncthreads();
    int pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        int xa = tmp[k], xb = tmp[NW + k];
        if (k < wid) {
            pa += xa;
            pb += xb;
        }
        sa += xa;
        sb += xb;
    }
    ea = pa + ia - a;
    eb = pb + ib - b;
    ta = sa;
    tb = sb;
    __syncthreads();  // tmp may be reused right after
}

// Fixed-order block sum of a float (wave butterflies, then wave partials in
// order).  `tmp` holds BLOCK/64 floats.  All threads call; all get the sum.
template <int BLOCK>
__device__ __forceinline__ float block_sum(float v, float *tmp)
{
    constexpr int NW = BLOCK / kWave;
    v = wave_sum(v);
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = v;
    __syncthreads();
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += tmp[k];
    __syncthreads();
    return s;
}

}  // namespace wc
