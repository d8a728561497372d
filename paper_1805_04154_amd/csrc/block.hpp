// Workgroup-wide scan/reduce helpers for 256-thread (4 x wave64) blocks.
#pragma once
#include "common.hpp"

namespace ps {

constexpr uint32_t kInf = 0xFFFFFFFFu;

// Exclusive suffix minimum over the block: min of v over all threads > tid.
__device__ __forceinline__ uint32_t block_excl_suffix_min(uint32_t v, uint32_t* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_down(incl, d);
        if (lane + d < 64) incl = min(incl, o);
    }
    uint32_t nxt = __shfl_down(incl, 1);
    if (lane == 63) nxt = kInf;
    if (lane == 0) sh[wid] = incl;
    __syncthreads();
    uint32_t tail = kInf;
    for (int w2 = wid + 1; w2 < kWaves; ++w2) tail = min(tail, sh[w2]);
    __syncthreads();
    return min(nxt, tail);
}

// Exclusive prefix sum over the block.
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* sh, uint32_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w2 = 0; w2 < kWaves; ++w2) {
        if (w2 < wid) before += sh[w2];
        all += sh[w2];
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}


// Exclusive prefix sum over a block of NW wave64s.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_sum_w(uint32_t v, uint32_t* sh, uint32_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) {
        const uint32_t t = sh[w2];
        before += (w2 < wid) ? t : 0u;
        all += t;
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}

// Exclusive prefix sum over the block for 64-bit values.
__device__ __forceinline__ uint64_t block_excl_sum64(uint64_t v, uint64_t* sh, uint64_t* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int w2 = 0; w2 < kWaves; ++w2) {
        if (w2 < wid) before += sh[w2];
        all += sh[w2];
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}

}  // namespace ps
