// pred.hip -- predecessor arrays read off finished distances: a BFS tree
// (Sec. 5.1) or a shortest-path tree (Sec. 5.2).  pred[src] = src, -1 where
// unreached, otherwise the first neighbour u in v's row that is one step
// closer to the source (depth[u] = depth[v] - 1, or dist[u] + w = dist[v]).
// Taking the first such neighbour in row order makes the result unique (the
// smallest id when rows are sorted) instead of whichever discoverer won a
// race during the traversal.
//
// Lane = vertex for rows of up to 64 entries, scanned four at a time with the
// loads issued together; longer rows are left to the whole wave, which scans
// 64 entries per step and takes the first hit with a ballot, so a hub whose
// first closer neighbour sits deep in its row costs (position / 64) steps.
#include "engine.h"

namespace gfr {

struct BfsCloser {
    const int32_t *d;
    __device__ bool reached(int32_t v, int64_t &kv) const
    {
        kv = d[v];
        return kv >= 0;
    }
    __device__ bool closer(int64_t kv, int32_t, int32_t u) const { return (int64_t)d[u] == kv - 1; }
};

struct SsspCloser {
    const uint32_t *d;
    const uint32_t *W;
    __device__ bool reached(int32_t v, int64_t &kv) const
    {
        kv = d[v];
        return d[v] != 0xFFFFFFFFu;
    }
    __device__ bool closer(int64_t kv, int32_t e, int32_t u) const
    {
        const uint32_t du = d[u];
        return (du != 0xFFFFFFFFu) & ((int64_t)du + (int64_t)W[e] == kv);
    }
};

template <class T>
__global__ __launch_bounds__(GFR_BLOCK) void pred_kernel(const int32_t *R, const int32_t *C, int32_t n, int32_t src,
                                                         T t, int32_t *pred)
{
    const int lane = lane_id();
    const uint32_t waves = gridDim.x * GFR_WAVES;
    for (uint32_t grp = blockIdx.x * GFR_WAVES + threadIdx.x / 64; grp * 64u < (uint32_t)n; grp += waves) {
        const int32_t v = (int32_t)(grp * 64u) + lane;
        int32_t p = -1;
        int64_t kv = 0;
        bool longrow = false;
        if (v < n && t.reached(v, kv)) {
            if (v == src) {
                p = src;
            } else {
                const int32_t rb = R[v], re = R[v + 1];
                if (re - rb > 64) {
                    longrow = true;
                } else {
                    for (int32_t e = rb; e < re; e += 4) {
                        const int32_t k = min(4, re - e);
                        int32_t u[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) u[j] = C[j < k ? e + j : e];
                        bool hit[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) hit[j] = (j < k) & t.closer(kv, j < k ? e + j : e, u[j]);
                        int32_t f = -1;
#pragma unroll
                        for (int j = 3; j >= 0; --j) f = hit[j] ? u[j] : f;
                        if (f >= 0) {
                            p = f;
                            break;
                        }
                    }
                }
            }
        }
        // long rows, one at a time by the whole wave
        uint64_t lm = ballot(longrow);
        while (lm) {
            const int j = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int32_t vj = (int32_t)(grp * 64u) + j;
            const int64_t kj = (int64_t)(int32_t)shfl_u32((uint32_t)kv, j) |
                               ((int64_t)shfl_u32((uint32_t)((uint64_t)kv >> 32), j) << 32);
            const int32_t rb = R[vj], re = R[vj + 1];
            int32_t found = -1;
            for (int32_t e0 = rb; e0 < re; e0 += 64) {
                const int32_t e = min(e0 + lane, re - 1);
                const int32_t u = C[e];
                const bool hit = (e0 + lane < re) & t.closer(kj, e, u);
                const uint64_t hm = ballot(hit);
                if (hm) {
                    found = (int32_t)shfl_u32((uint32_t)u, __ffsll((unsigned long long)hm) - 1);
                    break;
                }
            }
            if (lane == j) p = found;
        }
        if (v < n) pred[v] = p;
    }
}

void run_bfs_pred(Ctx &c, Graph &g, int32_t src, const int32_t *depth, int32_t *pred, hipStream_t s)
{
    hipLaunchKernelGGL(pred_kernel<BfsCloser>, dim3(grid_blocks(c, 4)), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(),
                       g.C.as<int32_t>(), g.n, src, BfsCloser{depth}, pred);
    GFR_LAUNCH_CHECK();
}

void run_sssp_pred(Ctx &c, Graph &g, int32_t src, const uint32_t *dist, int32_t *pred, hipStream_t s)
{
    hipLaunchKernelGGL(pred_kernel<SsspCloser>, dim3(grid_blocks(c, 4)), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(),
                       g.C.as<int32_t>(), g.n, src, SsspCloser{dist, g.W.as<uint32_t>()}, pred);
    GFR_LAUNCH_CHECK();
}

}  // namespace gfr
