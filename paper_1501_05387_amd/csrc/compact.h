// compact.h -- ordered frontier compaction (the filter's compaction step,
// Sec. 4.1 "Filter": scan-based culling and deduplication of the frontier).
//
// Advance kernels mark the next frontier in a byte array with plain stores
// (idempotent: several threads may store the same mark).  On MI355X scattered
// atomics are capped near 27 G ops/s at any table size while plain stores and
// loads run several times faster, so marking needs no atomics at all.
//
// This kernel turns the marks into the next frontier queue in vertex order.
// Every thread owns `wpt` consecutive groups of 32 vertices ("words"); the
// caller's functor reads (and consumes) the marks of a word and returns them
// as a 32-bit mask.  Pass 1 counts vertices and their degrees; a block scan
// and a decoupled look-back across work-groups give every thread its global
// slot and edge offset; pass 2 stages the group's entries in LDS and writes
// (vertex, edge offset, row start) contiguously, plus the chunk index used by
// the load-balanced advance.  No counter is shared by all work-groups (on
// MI355X same-address atomics serialise at ~11 ns each): the only
// cross-group traffic is one 64-bit status word per work-group, and the last
// work-group, which learns the grand totals, runs the caller's control.
//
// Status words (one per work-group, two parity buffers): flag in bits 62-63
// (1 = aggregate of this group, 2 = inclusive prefix), entry count in bits
// 31-61, edge count in bits 0-30.  Sums of packed values stay packed because
// entries < 2^31 and edges < 2^31.
//
// Marked vertices without edges are dropped from the queue (they have no work
// for the next advance and would break the one-entry-per-chunk-start rule).
#pragma once

#include "device.h"

namespace gfr {

constexpr unsigned long long ST_AGG = 1ull << 62;
constexpr unsigned long long ST_INC = 2ull << 62;
constexpr unsigned long long ST_FLAGS = 3ull << 62;
constexpr int COMPACT_MAX_WPT = 32;   // words per thread held in registers
constexpr int COMPACT_STAGE = 2048;   // entries staged in LDS per output round
constexpr int COMPACT_EPT = COMPACT_STAGE / GFR_BLOCK;

// Status words carry their whole payload, and no other data written by a
// predecessor group is read by its successors, so relaxed device-coherent
// atomics suffice.  (Acquire/release at device scope would write back or
// invalidate the caches on every access, which a spinning look-back repeats.)
__device__ __forceinline__ unsigned long long st_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_store(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 32 mark bytes (each 0 or 1) at p -> 32-bit mask; p is 32-byte aligned
__device__ __forceinline__ uint32_t marks_to_mask(const uint8_t *p)
{
    const uint4 a = *(const uint4 *)p, b = *(const uint4 *)(p + 16);
    const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // bytes of value 0/1 at bit positions 0,8,16,24 -> bits 21..24 of the product
        const uint32_t y = x[i] & 0x01010101u;
        m |= ((y * 0x00204081u) >> 21 & 0xFu) << (4 * i);
    }
    return m;
}

__device__ __forceinline__ void clear_marks(uint8_t *p)
{
    *(uint4 *)p = make_uint4(0, 0, 0, 0);
    *(uint4 *)(p + 16) = make_uint4(0, 0, 0, 0);
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

// exclusive block scan; *total receives the block sum
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long x, unsigned long long *total)
{
    __shared__ unsigned long long s_w[GFR_WAVES];
    const int w = threadIdx.x / 64;
    const unsigned long long inc = wave_incl_scan_u64(x);
    __syncthreads();
    if (lane_id() == 63) s_w[w] = inc;
    __syncthreads();
    unsigned long long base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < GFR_WAVES; ++i) {
        if (i < w) base += s_w[i];
        tot += s_w[i];
    }
    *total = tot;
    return base + inc - x;
}

// Work-group exclusive prefix by decoupled look-back (wave 0; the other waves
// receive it through LDS).  Every wait is bounded, so the kernel always ends;
// if a bound is ever exhausted *err is set and the results are flagged bad.
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

// Keep only the vertices of `bits` (vertices 32w+b) that have edges, and
// return the sum of their degrees.  The 33 row offsets are fetched with
// independent loads (vector loads when the run lies inside R), so the latency
// is paid once per word, not once per vertex.
__device__ __forceinline__ uint32_t word_degrees(const int32_t *R, int32_t n, uint32_t w, uint32_t &bits)
{
    const int32_t v0 = (int32_t)(w * 32u);
    int32_t r[33];
    if (v0 + 32 <= n) {
        const int4 *p = (const int4 *)(R + v0);   // R + 32w is 128-byte aligned
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int4 x = p[i];
            r[4 * i] = x.x;
            r[4 * i + 1] = x.y;
            r[4 * i + 2] = x.z;
            r[4 * i + 3] = x.w;
        }
        r[32] = R[v0 + 32];
    } else {
#pragma unroll
        for (int i = 0; i < 33; ++i) r[i] = (v0 + i <= n) ? R[v0 + i] : r[i > 0 ? i - 1 : 0];
    }
    uint32_t s = 0, keep = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const uint32_t d = (uint32_t)(r[i + 1] - r[i]);
        if (((bits >> i) & 1u) && d) {
            s += d;
            keep |= 1u << i;
        }
    }
    bits = keep;
    return s;
}

// Degrees of the marked vertices of word w when every thread owns one word
// (a wave's 64 words are then consecutive).  A full wave whose words hold at
// least 8 marked vertices a word on average, all below n, reads the 2,049 row
// offsets of its run with coalesced 16-byte loads into LDS and takes its
// 33-entry slices from there (offset j at j + j/32, so that the lanes' slices
// fall in different banks), instead of 33 offsets a lane 128 bytes apart.
// Otherwise as word_degrees.  s_r: this wave's 2,113 LDS words (one run per
// wave and launch).
constexpr int COMPACT_RUN_LDS = 2 * 1024 + 64 + 1;

__device__ __forceinline__ uint32_t run_degrees(const int32_t *R, int32_t n, uint32_t w, bool active, uint32_t &bits,
                                                int32_t *s_r)
{
    if (ballot(active) == ~0ull) {
        const uint32_t wfirst = (uint32_t)__builtin_amdgcn_readfirstlane((int)w);
        const uint32_t tot = wave_sum_u32(__popc(bits));
        if (tot >= 64u * 8u && (wfirst + 64ull) * 32ull <= (unsigned long long)n) {
            const int l = lane_id();
            const int4 *p = (const int4 *)(R + 32ull * wfirst);   // 128-byte aligned
            int4 x[8];
#pragma unroll
            for (int it = 0; it < 8; ++it) x[it] = p[it * 64 + l];
            const int32_t last = R[32ull * wfirst + 2048];   // R has n + 1 entries
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                const int j = 4 * (it * 64 + l), pj = j + j / 32;   // four offsets in one 32-block
                s_r[pj] = x[it].x;
                s_r[pj + 1] = x[it].y;
                s_r[pj + 2] = x[it].z;
                s_r[pj + 3] = x[it].w;
            }
            if (l == 0) s_r[2048 + 64] = last;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // offsets 32l .. 32l + 32 sit at 33l .. 33l + 31 and 33(l + 1)
            uint32_t sum = 0, keep = 0;
            int32_t prev = s_r[33 * l];
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const int32_t next = s_r[i == 31 ? 33 * l + 33 : 33 * l + i + 1];
                const uint32_t d = (uint32_t)(next - prev);
                if (((bits >> i) & 1u) && d) {
                    sum += d;
                    keep |= 1u << i;
                }
                prev = next;
            }
            bits = keep;
            return sum;
        }
    }
    return (active && bits) ? word_degrees(R, n, w, bits) : 0u;
}

// Compaction kernel.  M: functor with
//     bool skip() const                  whole launch is a no-op (uniform)
//     uint32_t mask(uint32_t w)          marks of vertices 32w..32w+31 (may consume / update state)
//     void partial(uint32_t cnt)         called by every thread before the group publishes; side
//                                        results it sends to the last group need their own fence
//     void control(uint32_t nf, uint32_t mf)  called by every thread of the last group
template <class M>
__global__ __launch_bounds__(GFR_BLOCK) void compact_kernel(const int32_t *R, int32_t n, uint32_t nwords,
                                                            uint32_t wpt, M mk, FrontierQ q, uint32_t chunk,
                                                            unsigned long long *status2, const uint32_t *parity,
                                                            uint32_t *err)
{
    if (mk.skip()) return;
    const uint32_t p = *parity;
    unsigned long long *status = status2 + (size_t)p * gridDim.x;
    const uint32_t w0 = (blockIdx.x * GFR_BLOCK + threadIdx.x) * wpt;
    uint32_t words[COMPACT_MAX_WPT];
    uint32_t cnt = 0, edges = 0;
#pragma unroll
    for (int i = 0; i < COMPACT_MAX_WPT; ++i) words[i] = 0;
    if (wpt == 1) {
        __shared__ int32_t s_run[GFR_WAVES][COMPACT_RUN_LDS];
        const bool active = w0 < nwords;
        uint32_t bits = active ? mk.mask(w0) : 0u;
        edges = run_degrees(R, n, w0, active, bits, s_run[threadIdx.x / 64]);   // drops vertices without edges
        cnt = __popc(bits);
        words[0] = bits;
    } else {
#pragma unroll
        for (int i = 0; i < COMPACT_MAX_WPT; ++i) {
            if ((uint32_t)i < wpt && w0 + i < nwords) {
                uint32_t bits = mk.mask(w0 + i);
                if (bits) {
                    edges += word_degrees(R, n, w0 + i, bits);   // drops vertices without edges
                    cnt += __popc(bits);
                }
                words[i] = bits;
            }
        }
    }
    mk.partial(cnt);
    unsigned long long btot;
    const unsigned long long mine = ((unsigned long long)cnt << 31) | edges;
    const unsigned long long excl = block_excl_scan_u64(mine, &btot);
    const unsigned long long base = lookback_prefix(status, btot, err);
    const uint32_t bcnt = (uint32_t)(btot >> 31);
    const uint32_t slot0 = (uint32_t)(base >> 31);
    uint32_t eoff = (uint32_t)(base & 0x7FFFFFFFull);   // edge offset of the next staged entry

    // pass 2: stage entries in LDS round by round, write them contiguously
    __shared__ int32_t s_v[COMPACT_STAGE];
    __shared__ uint32_t s_e[GFR_WAVES];
    uint32_t my = (uint32_t)(excl >> 31);   // block-local index of this thread's next entry
    int wi = 0;
    uint32_t cur = words[0];
    for (uint32_t r0 = 0; r0 < bcnt; r0 += COMPACT_STAGE) {
        const uint32_t r1 = r0 + COMPACT_STAGE;
        // this thread's entries falling into [r0, r1)
        while (my < r1 && wi < (int)wpt) {
            if (!cur) {
                if (++wi < (int)wpt) {
#pragma unroll
                    for (int i = 1; i < COMPACT_MAX_WPT; ++i)
                        if (i == wi) cur = words[i];
                }
                continue;
            }
            const int bi = __ffs(cur) - 1;
            cur &= cur - 1;
            s_v[my - r0] = (int32_t)((w0 + wi) * 32u) + bi;
            ++my;
        }
        __syncthreads();
        const uint32_t cntr = min((uint32_t)COMPACT_STAGE, bcnt - r0);
        // each thread takes COMPACT_EPT consecutive staged entries
        const uint32_t j0 = threadIdx.x * COMPACT_EPT;
        int32_t vv[COMPACT_EPT], rr[COMPACT_EPT];
        uint32_t dd[COMPACT_EPT], tsum = 0;
#pragma unroll
        for (int k = 0; k < COMPACT_EPT; ++k) {
            dd[k] = 0;
            vv[k] = 0;
            rr[k] = 0;
            if (j0 + k < cntr) {
                vv[k] = s_v[j0 + k];
                rr[k] = R[vv[k]];
                dd[k] = (uint32_t)(R[vv[k] + 1] - rr[k]);
                tsum += dd[k];
            }
        }
        // exclusive scan of the per-thread degree sums
        uint32_t inc = wave_incl_scan(tsum);
        if (lane_id() == 63) s_e[threadIdx.x / 64] = inc;
        __syncthreads();
        uint32_t before = 0, rtot = 0;
#pragma unroll
        for (int i = 0; i < GFR_WAVES; ++i) {
            if (i < (int)(threadIdx.x / 64)) before += s_e[i];
            rtot += s_e[i];
        }
        uint32_t o = eoff + before + inc - tsum;
#pragma unroll
        for (int k = 0; k < COMPACT_EPT; ++k) {
            if (j0 + k < cntr) {
                const uint32_t slot = slot0 + r0 + j0 + k;
                q.v[slot] = vv[k];
                q.off[slot] = o;
                q.row[slot] = rr[k];
                for (uint32_t c = (o + chunk - 1) / chunk; (uint64_t)c * chunk < (uint64_t)o + dd[k]; ++c)
                    q.part[c] = (int32_t)slot;
                o += dd[k];
            }
        }
        eoff += rtot;
        __syncthreads();
    }
    // clear this group's slot of the other parity for the next launch
    if (threadIdx.x == 0) status2[(size_t)(p ^ 1u) * gridDim.x + blockIdx.x] = 0ull;
    if (blockIdx.x == gridDim.x - 1) {   // whole group: control may reduce per-group partials
        __atomic_thread_fence(__ATOMIC_ACQUIRE);   // see the side results of partial()
        const unsigned long long all = base + btot;
        mk.control((uint32_t)(all >> 31), (uint32_t)(all & 0x7FFFFFFFull));
    }
}

// launch geometry for nwords words of 32 vertices: two work-groups per CU
// (measured on R-MAT s22: single-source BFS 0.38 -> 0.33 ms against one per
// CU, batched steps unchanged, four per CU slower), and no more work-groups
// than there are words for one word per thread (a small graph keeps its
// look-back chain short)
struct CompactGeom {
    uint32_t blocks, wpt;
};

static inline CompactGeom compact_geom(uint32_t nwords, int num_cu)
{
    CompactGeom g;
    g.blocks = 2u * (uint32_t)num_cu;
    const uint32_t needed = (uint32_t)(((uint64_t)nwords + GFR_BLOCK - 1) / GFR_BLOCK);
    if (needed < g.blocks) g.blocks = needed < 1u ? 1u : needed;
    const uint64_t threads = (uint64_t)g.blocks * GFR_BLOCK;
    g.wpt = (uint32_t)((nwords + threads - 1) / threads);
    if (g.wpt < 1) g.wpt = 1;
    if (g.wpt > (uint32_t)COMPACT_MAX_WPT) {
        g.wpt = COMPACT_MAX_WPT;
        g.blocks = (uint32_t)((nwords + (uint64_t)GFR_BLOCK * COMPACT_MAX_WPT - 1) /
                              ((uint64_t)GFR_BLOCK * COMPACT_MAX_WPT));
    }
    return g;
}

}  // namespace gfr
