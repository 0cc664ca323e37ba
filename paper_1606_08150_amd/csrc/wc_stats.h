// Per-call work counters: each thread accumulates in registers; at the end of a
// kernel the block reduces them (wave sums, then LDS) and adds them to one
// replica of the device counters with a single atomic per counter.
#pragma once

#include "wc_device.h"
#include "wc_internal.h"

namespace wc {

// 32-bit per thread: a thread's share of one kernel's work is bounded by the
// int32 edge and vertex counts of the CSR; the block sums are 64-bit.
struct StatAcc {
    unsigned int items = 0, dispatches = 0, edges = 0, buffered = 0, updates = 0, updates_buffered = 0;
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// All threads of the block must call this (it contains barriers).
__device__ __forceinline__ void stat_flush(DevStats *s, const StatAcc &acc)
{
    constexpr int K = 6;
    __shared__ unsigned long long sh[K];
    if (threadIdx.x < K) sh[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long v[K] = {acc.items, acc.dispatches, acc.edges, acc.buffered, acc.updates,
                               acc.updates_buffered};
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_u64(v[k]);
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (v[k]) atomicAdd(&sh[k], v[k]);
    }
    __syncthreads();
    if (threadIdx.x < K && sh[threadIdx.x]) {
        StatRep &r = s->rep[blockIdx.x % kStatReps];
        unsigned long long *dst[K] = {&r.items_buffered,  &r.dispatches, &r.edges_processed,
                                      &r.edges_buffered,  &r.updates,    &r.updates_buffered};
        atomic_add_dev(dst[threadIdx.x], sh[threadIdx.x]);
    }
}

// Publishes `value` to entry `index` of the context's host ring, tagged with
// the current call's epoch (set in the counters by the call's first kernel).
// One 64-bit system-scope store, so the host sees tag and value together.
__device__ __forceinline__ void publish_host(unsigned long long *ring, int index, const DevStats *s, int value)
{
    const unsigned long long word = ((unsigned long long)s->epoch << 32) | (unsigned long long)(unsigned int)value;
    __hip_atomic_store(&ring[index], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace wc
