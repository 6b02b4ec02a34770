// cc.hip -- connected components by hooking and pointer jumping (Sec. 5.4).
//
// label[] is a forest of parent pointers with label[v] <= v.  A hooking round
// walks an edge frontier: for an edge (a,b) whose endpoints carry different
// labels la, lb, the larger label is hooked under the smaller one with
// atomicMin; the filter of Sec. 5.4 is fused in, keeping only edges whose
// endpoints disagreed.  Pointer jumping then flattens every tree to a star.
// Rounds repeat until an edge frontier comes back empty.  Because every hook
// moves a label to a smaller id of the same component, the root that survives
// is the component's smallest vertex id, the label convention of this library.
//
// Round 1 hooks over the full CSR (each undirected edge once, a < b), round 2
// sweeps the full CSR again and compacts the disagreeing edges into a list,
// later rounds work on that list only.
#include "engine.h"
#include "gather.h"

namespace gfr {

struct CcCtl {
    uint32_t kept;      // edges appended to the out list this round
    uint32_t roots;
};

__device__ __forceinline__ void hook(int32_t *label, int32_t la, int32_t lb)
{
    if (la < lb) atomicMin(label + lb, la);
    else atomicMin(label + la, lb);
}

// wave-aggregated append of an edge pair
__device__ __forceinline__ void wave_append_pair(bool valid, int32_t a, int32_t b, uint32_t *count, int2 *out)
{
    const uint64_t mask = ballot(valid);
    if (mask == 0) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = shfl_u32(base, leader);
    if (valid) out[base + lanes_below(mask)] = make_int2(a, b);
}

struct HookOp {
    int32_t *label;
    int2 *out;        // null: do not compact
    uint32_t *count;
    __device__ void operator()(bool valid, int32_t b, int32_t a) const
    {
        bool keep = false;
        if (valid && a < b) {
            const int32_t la = label[a], lb = label[b];
            if (la != lb) {
                hook(label, la, lb);
                keep = true;
            }
        }
        if (out) wave_append_pair(keep, a, b, count, out);
    }
};

__global__ void cc_init(int32_t *label, int32_t n)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) label[v] = v;
}

__global__ __launch_bounds__(GFR_BLOCK) void cc_jump(int32_t *label, int32_t n)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int32_t r = label[v];
        if (r == v) continue;
        int32_t p = label[r];
        while (p != r) {
            r = p;
            p = label[r];
        }
        label[v] = r;
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void cc_hook_list(int32_t *label, const int2 *in, const uint32_t *nin,
                                                           int2 *out, uint32_t *nout)
{
    const uint32_t cnt = *nin;
    for (uint32_t base = blockIdx.x * GFR_BLOCK; base < cnt; base += gridDim.x * GFR_BLOCK) {
        const uint32_t i = base + threadIdx.x;
        bool keep = false;
        int2 e = make_int2(0, 0);
        if (i < cnt) {
            e = in[i];
            const int32_t la = label[e.x], lb = label[e.y];
            if (la != lb) {
                hook(label, la, lb);
                keep = true;
            }
        }
        wave_append_pair(keep, e.x, e.y, nout, out);
    }
}

// per-group root counts (plain stores), summed by cc_sum
__global__ __launch_bounds__(GFR_BLOCK) void cc_count_roots(const int32_t *label, int32_t n, uint32_t *part)
{
    uint32_t r = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        r += (label[v] == v);
    __shared__ uint32_t s[GFR_WAVES];
    r = wave_sum_u32(r);
    if (lane_id() == 0) s[threadIdx.x / 64] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < GFR_WAVES; ++i) t += s[i];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void cc_sum(const uint32_t *part, uint32_t nparts, uint32_t *out)
{
    uint32_t r = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) r += part[i];
    __shared__ uint32_t s[GFR_WAVES];
    r = wave_sum_u32(r);
    if (lane_id() == 0) s[threadIdx.x / 64] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < GFR_WAVES; ++i) t += s[i];
        *out = t;
    }
}

void run_cc(Ctx &c, Graph &g, int32_t *label, int32_t *ncomp, hipStream_t s)
{
    const int32_t n = g.n;
    const size_t cap = (size_t)(g.m / 2) + 1;
    const int G = grid_blocks(c, 4);
    c.arena.reserve(2 * al256(8 * cap) + al256(4 * 64) + al256(4ull * G));
    int2 *list[2] = {c.arena.take<int2>(cap), c.arena.take<int2>(cap)};
    uint32_t *ctr = c.arena.take<uint32_t>(64);   // [round] kept counters, [63] roots
    uint32_t *rpart = c.arena.take<uint32_t>(G);
    fill_u32(ctr, 0u, 64, s);
    hipLaunchKernelGGL(cc_init, dim3(G), dim3(GFR_BLOCK), 0, s, label, n);
    const int32_t *C = g.C.as<int32_t>();
    // round 1: hook over the full CSR, no compaction
    hipLaunchKernelGGL((for_each_edge<GATHER_CH, HookOp>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full, g.full_counts,
                       g.full_counts + 1, C, HookOp{label, nullptr, nullptr});
    hipLaunchKernelGGL(cc_jump, dim3(G), dim3(GFR_BLOCK), 0, s, label, n);
    // round 2: sweep the full CSR again, keep disagreeing edges
    hipLaunchKernelGGL((for_each_edge<GATHER_CH, HookOp>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full, g.full_counts,
                       g.full_counts + 1, C, HookOp{label, list[0], ctr + 0});
    hipLaunchKernelGGL(cc_jump, dim3(G), dim3(GFR_BLOCK), 0, s, label, n);
    GFR_LAUNCH_CHECK();
    int rounds = 2;
    uint32_t kept = 0;
    for (int r = 0;; ++r) {
        GFR_HIP(hipMemcpyAsync(c.pinned, ctr + (r % 62), 4, hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        kept = c.pinned[0];
        if (kept == 0) break;
        if (rounds > 2 * 64 + 40) fail(GFR_E_DEVICE, "cc: hooking did not converge");
        uint32_t *nxt = ctr + ((r + 1) % 62);
        fill_u32(nxt, 0u, 1, s);
        hipLaunchKernelGGL(cc_hook_list, dim3(G), dim3(GFR_BLOCK), 0, s, label, list[r & 1], ctr + (r % 62),
                           list[(r + 1) & 1], nxt);
        hipLaunchKernelGGL(cc_jump, dim3(G), dim3(GFR_BLOCK), 0, s, label, n);
        GFR_LAUNCH_CHECK();
        ++rounds;
    }
    hipLaunchKernelGGL(cc_count_roots, dim3(G), dim3(GFR_BLOCK), 0, s, label, n, rpart);
    hipLaunchKernelGGL(cc_sum, dim3(1), dim3(GFR_BLOCK), 0, s, rpart, (uint32_t)G, ctr + 63);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, ctr + 63, 4, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    *ncomp = (int32_t)c.pinned[0];
    c.stats.v["rounds"] = rounds;
}

}  // namespace gfr
