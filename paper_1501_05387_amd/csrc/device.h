// device.h -- wave-level building blocks shared by the engine's HIP kernels.
//
// gfx950 executes 64-lane wavefronts; every helper here assumes the whole
// wave calls it in converged control flow (all 64 lanes active).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GFR_BLOCK 256                 // work-group size used by every traversal kernel
#define GFR_WAVES (GFR_BLOCK / 64)

namespace gfr {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// number of set bits of `mask` in lanes below the calling lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t shfl_u32(uint32_t x, int src) { return (uint32_t)__shfl((int)x, src, 64); }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src)
{
    uint32_t lo = shfl_u32((uint32_t)x, src), hi = shfl_u32((uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// inclusive prefix sum across the wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += (uint32_t)__shfl_xor((int)x, d, 64);
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, d, 64);
        uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), d, 64);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x |= (uint32_t)__shfl_xor((int)x, d, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t y = (uint32_t)__shfl_xor((int)x, d, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Butterfly sum: a fixed pairwise (tree) order, identical on every call.
__device__ __forceinline__ float wave_sum_f32(float x)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// A frontier queue whose entries carry the exclusive prefix sum of their
// degrees (off), their CSR row start (row) and a chunk index (part): part[c]
// is the entry holding edge c*chunk of the concatenated neighbour lists.
// Entries with degree zero are never stored, so every chunk start falls
// inside exactly one entry.
struct FrontierQ {
    int32_t *v;
    uint32_t *off;
    int32_t *row;
    int32_t *part;
};

// Largest i in [lo, hi] with a[i] <= key (a sorted ascending, a[lo] <= key).
__device__ __forceinline__ int upper_index(const uint32_t *a, int lo, int hi, uint32_t key)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace gfr
