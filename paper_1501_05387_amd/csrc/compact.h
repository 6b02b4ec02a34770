// compact.h -- ordered bitmap -> frontier-queue compaction (the filter's
// compaction step, Sec. 4.1 "Filter": scan-based culling of the frontier).
//
// Advance kernels only set bits in a frontier bitmap (many threads, distinct
// words).  This kernel turns the bitmap into the next frontier queue in vertex
// order: every thread owns a run of consecutive bitmap words, counts its
// vertices and their degrees, a block scan and a decoupled look-back across
// work-groups give every run its global slot and edge offset, and a second
// pass over the same words writes (vertex, edge offset, row start) plus the
// chunk index of the load-balanced advance.
//
// No counter is shared by all work-groups: on MI355X same-address atomics from
// hundreds of work-groups serialise at the memory side, so the only
// cross-group traffic is one 64-bit status word per work-group.  The last
// work-group knows the grand totals and runs the caller's per-level control.
//
// Status words (one per work-group, two parity buffers): flag in bits 62-63
// (1 = aggregate of this group, 2 = inclusive prefix), entry count in bits
// 31-61, edge count in bits 0-30.  Sums of packed values stay packed because
// entries < 2^31 and edges < 2^31.
#pragma once

#include "device.h"

namespace gfr {

constexpr unsigned long long ST_AGG = 1ull << 62;
constexpr unsigned long long ST_INC = 2ull << 62;
constexpr unsigned long long ST_FLAGS = 3ull << 62;
constexpr int COMPACT_MAX_WPT = 32;   // bitmap words per thread held in registers

__device__ __forceinline__ unsigned long long st_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_store(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long x)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
        if (l >= d) x += ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// exclusive block scan of packed values; *total receives the block sum
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long x, unsigned long long *total)
{
    __shared__ unsigned long long s_w[GFR_WAVES];
    const int w = threadIdx.x / 64;
    const unsigned long long inc = wave_incl_scan_u64(x);
    if (lane_id() == 63) s_w[w] = inc;
    __syncthreads();
    unsigned long long base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < GFR_WAVES; ++i) {
        if (i < w) base += s_w[i];
        tot += s_w[i];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

// Work-group exclusive prefix by decoupled look-back (wave 0 only; the other
// waves receive it through LDS).  `spin_budget` bounds every wait so the
// kernel always terminates; on exhaustion *err is set and 0 is used.
__device__ __forceinline__ unsigned long long lookback_prefix(unsigned long long *status, unsigned long long agg,
                                                              uint32_t *err)
{
    __shared__ unsigned long long s_prefix;
    const int b = blockIdx.x;
    if (threadIdx.x < 64) {
        const int lane = lane_id();
        if (b == 0) {
            if (lane == 0) {
                st_store(status, ST_INC | agg);
                s_prefix = 0;
            }
        } else {
            if (lane == 0) st_store(status + b, ST_AGG | agg);
            unsigned long long prefix = 0;
            int top = b - 1;   // next predecessor to inspect
            uint32_t budget = 1u << 24;
            for (;;) {
                const int j = top - lane;
                unsigned long long st = j >= 0 ? st_load(status + j) : ST_INC;
                // wait until every lane of the window sees a published value
                while (ballot((st & ST_FLAGS) == 0) != 0) {
                    if ((st & ST_FLAGS) == 0) st = st_load(status + j);
                    if (--budget == 0) break;
                }
                if (budget == 0) {
                    if (lane == 0) *err = 1u;
                    prefix = 0;
                    break;
                }
                const uint64_t inc_mask = ballot((st & ST_FLAGS) == ST_INC);
                const int stop = inc_mask ? (__ffsll((unsigned long long)inc_mask) - 1) : 64;
                unsigned long long v = lane <= stop ? (st & ~ST_FLAGS) : 0ull;
                // sum over lanes (order irrelevant: integers)
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) {
                    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, 64);
                    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, 64);
                    v += ((unsigned long long)hi << 32) | lo;
                }
                prefix += v;
                if (stop < 64) break;
                top -= 64;
            }
            if (lane == 0) {
                st_store(status + b, ST_INC | (prefix + agg));
                s_prefix = prefix;
            }
        }
    }
    __syncthreads();
    return s_prefix;
}

// Compaction kernel.  Words: functor with
//     bool skip() const                       -- whole launch is a no-op (uniform)
//     uint32_t get(uint32_t w) const          -- frontier bits of word w (may consume/modify state)
//     void partial(uint32_t cnt)              -- called by every thread before the group publishes
//                                                (may reduce per-thread side results)
//     void control(uint32_t nf, uint32_t mf)  -- called by every thread of the last group with the totals
// Every thread owns `wpt` consecutive words starting at (block*256 + thread)*wpt.
template <class Words>
__global__ __launch_bounds__(GFR_BLOCK) void compact_kernel(const int32_t *R, int32_t n, uint32_t nwords,
                                                            uint32_t wpt, Words W, FrontierQ q, uint32_t chunk,
                                                            unsigned long long *status2, const uint32_t *parity,
                                                            uint32_t *err)
{
    if (W.skip()) return;
    const uint32_t p = *parity;
    unsigned long long *status = status2 + (size_t)p * gridDim.x;
    const uint32_t w0 = (blockIdx.x * GFR_BLOCK + threadIdx.x) * wpt;
    uint32_t words[COMPACT_MAX_WPT];
    uint32_t cnt = 0, edges = 0;
#pragma unroll
    for (int i = 0; i < COMPACT_MAX_WPT; ++i) {
        words[i] = 0;
        if ((uint32_t)i < wpt && w0 + i < nwords) {
            uint32_t bits = W.get(w0 + i);
            words[i] = bits;
            while (bits) {
                const int bi = __ffs(bits) - 1;
                bits &= bits - 1;
                const int32_t v = (int32_t)((w0 + i) * 32u) + bi;
                if (v >= n) break;
                const int32_t d = R[v + 1] - R[v];
                if (d > 0) {
                    ++cnt;
                    edges += (uint32_t)d;
                }
            }
        }
    }
    W.partial(cnt);
    unsigned long long tot;
    const unsigned long long mine = ((unsigned long long)cnt << 31) | edges;
    const unsigned long long excl = block_excl_scan_u64(mine, &tot);
    const unsigned long long base = lookback_prefix(status, tot, err);
    uint32_t slot = (uint32_t)((base + excl) >> 31);
    uint32_t off = (uint32_t)((base + excl) & 0x7FFFFFFFull);
#pragma unroll
    for (int i = 0; i < COMPACT_MAX_WPT; ++i) {
        uint32_t bits = words[i];
        while (bits) {
            const int bi = __ffs(bits) - 1;
            bits &= bits - 1;
            const int32_t v = (int32_t)((w0 + i) * 32u) + bi;
            if (v >= n) break;
            const int32_t r0 = R[v], d = R[v + 1] - r0;
            if (d > 0) {
                q.v[slot] = v;
                q.off[slot] = off;
                q.row[slot] = r0;
                for (uint32_t c = (off + chunk - 1) / chunk; (uint64_t)c * chunk < (uint64_t)off + (uint32_t)d; ++c)
                    q.part[c] = (int32_t)slot;
                ++slot;
                off += (uint32_t)d;
            }
        }
    }
    // clear this group's slot of the other parity for the next launch
    if (threadIdx.x == 0) status2[(size_t)(p ^ 1u) * gridDim.x + blockIdx.x] = 0ull;
    if (blockIdx.x == gridDim.x - 1) {   // whole group: control may reduce per-group partials
        const unsigned long long all = base + tot;
        W.control((uint32_t)(all >> 31), (uint32_t)(all & 0x7FFFFFFFull));
    }
}

// launch geometry for a bitmap of nwords words
struct CompactGeom {
    uint32_t blocks, wpt;
};

static inline CompactGeom compact_geom(uint32_t nwords, int num_cu)
{
    CompactGeom g;
    g.blocks = (uint32_t)num_cu;
    const uint64_t threads = (uint64_t)g.blocks * GFR_BLOCK;
    g.wpt = (uint32_t)((nwords + threads - 1) / threads);
    if (g.wpt < 1) g.wpt = 1;
    if (g.wpt > (uint32_t)COMPACT_MAX_WPT) {
        g.wpt = COMPACT_MAX_WPT;
        g.blocks = (uint32_t)((nwords + (uint64_t)GFR_BLOCK * COMPACT_MAX_WPT - 1) / ((uint64_t)GFR_BLOCK * COMPACT_MAX_WPT));
    }
    return g;
}

}  // namespace gfr
