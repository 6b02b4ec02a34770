// gather.h -- load-balanced segmented gather-reduce over a frontier queue.
//
// For every entry i of a FrontierQ (vertex v_i, neighbour list starting at
// row_i, edge offset off_i in the concatenated lists) compute
//     S_i = sum over the neighbours u of v_i, in CSR order, of op(u, v_i)
// in FP64, then call fin(v_i, S_i) exactly once.  This is the advance step of
// Sec. 4.1 with a fused "compute" (Sec. 4.3), in the load-balanced
// partitioning form of Sec. 4.4: each work-group takes an equal slice of
// edges, so one hub's list is spread over many work-groups while short lists
// are packed together.
//
// Within a chunk the op values are staged in LDS; short segments are summed by
// one lane, long ones by a whole wave (64 strided partial sums combined by a
// butterfly).  Lists that cross chunk boundaries leave partial sums that a
// second, tiny kernel combines in chunk order.  For a fixed queue layout every
// sum is formed in a fixed order, so results are reproducible run to run.
#pragma once

#include "device.h"

namespace gfr {

struct GatherScratch {
    double *pfirst;   // per chunk: partial of the entry continuing into it
    double *plast;    // per chunk: partial of the entry starting in it and continuing out
};

template <int CH, class Op, class Fin>
__global__ __launch_bounds__(GFR_BLOCK) void gather_chunks(FrontierQ q, const uint32_t *nf_p,
                                                           const uint32_t *mf_p, const int32_t *C,
                                                           Op op, Fin fin, GatherScratch gs,
                                                           const uint32_t *stop)
{
    if (*stop) return;
    const uint32_t nf = *nf_p, mf = *mf_p;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    __shared__ uint32_t s_off[CH + 2];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    __shared__ double s_val[CH];
    __shared__ int32_t s_long[CH + 1];
    __shared__ int32_t s_nlong;
    const int wave = threadIdx.x / 64, lane = lane_id();
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t e0 = c * CH;
        const uint32_t e1 = min(e0 + (uint32_t)CH, mf);
        const int s = q.part[c];
        const int t = (c + 1 < nchunks) ? q.part[c + 1] : (int)nf - 1;
        const int cnt = t - s + 1;
        __syncthreads();
        if (threadIdx.x == 0) s_nlong = 0;
        for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            s_off[i] = q.off[s + i];
            s_row[i] = q.row[s + i];
            s_v[i] = q.v[s + i];
        }
        if (threadIdx.x == 0) s_off[cnt] = (t + 1 < (int)nf) ? q.off[t + 1] : mf;
        __syncthreads();
        {
            // every lane takes CH / GFR_BLOCK edges and issues all their column
            // loads, then all their value loads, before storing any value: the
            // loads of one lane overlap instead of waiting one after another.
            // Lanes past the chunk's end repeat its last edge (in bounds) and
            // store nothing.
            constexpr int EPT = CH / GFR_BLOCK;
            static_assert(CH % GFR_BLOCK == 0, "chunk must be a multiple of the work-group size");
            int ii[EPT];
            int32_t u[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const uint32_t e = min(e0 + (uint32_t)(j * GFR_BLOCK) + threadIdx.x, e1 - 1u);
                ii[j] = upper_index(s_off, 0, cnt - 1, e);
                u[j] = C[s_row[ii[j]] + (int32_t)(e - s_off[ii[j]])];
            }
            double val[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) val[j] = op(u[j], s_v[ii[j]]);
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const uint32_t k = (uint32_t)(j * GFR_BLOCK) + threadIdx.x;
                if (k < e1 - e0) s_val[k] = val[j];
            }
        }
        __syncthreads();
        // short segments: one lane each; long ones are queued for the waves
        for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            const uint32_t a = max(s_off[i], e0), b = min(s_off[i + 1], e1);
            if (b <= a) continue;  // list starts exactly at the next chunk
            if (b - a <= 32u) {
                double acc = 0.0;
                for (uint32_t j = a; j < b; ++j) acc += s_val[j - e0];
                const bool starts = s_off[i] >= e0, ends = s_off[i + 1] <= e1;
                if (starts && ends) fin(s_v[i], acc);
                else if (!starts) gs.pfirst[c] = acc;
                else gs.plast[c] = acc;
            } else {
                s_long[atomicAdd(&s_nlong, 1)] = i;
            }
        }
        __syncthreads();
        const int nl = s_nlong;
        for (int li = wave; li < nl; li += GFR_WAVES) {
            const int i = s_long[li];
            const uint32_t a = max(s_off[i], e0), b = min(s_off[i + 1], e1);
            double acc = 0.0;
            for (uint32_t j = a + lane; j < b; j += 64) acc += s_val[j - e0];
            acc = wave_sum_f64(acc);
            if (lane == 0) {
                const bool starts = s_off[i] >= e0, ends = s_off[i + 1] <= e1;
                if (starts && ends) fin(s_v[i], acc);
                else if (!starts) gs.pfirst[c] = acc;
                else gs.plast[c] = acc;
            }
        }
    }
}

// One lane per chunk: if the chunk's last entry starts in it and continues
// past its end, add the partials of the following chunks in order.
template <int CH, class Fin>
__global__ __launch_bounds__(GFR_BLOCK) void gather_fixup(FrontierQ q, const uint32_t *nf_p,
                                                          const uint32_t *mf_p, Fin fin,
                                                          GatherScratch gs, const uint32_t *stop)
{
    if (*stop) return;
    const uint32_t nf = *nf_p, mf = *mf_p;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    for (uint32_t c = blockIdx.x * GFR_BLOCK + threadIdx.x; c < nchunks; c += gridDim.x * GFR_BLOCK) {
        const uint32_t e0 = c * CH, e1 = min(e0 + (uint32_t)CH, mf);
        const int t = (c + 1 < nchunks) ? q.part[c + 1] : (int)nf - 1;
        const uint32_t ot = q.off[t];
        const uint32_t endt = (t + 1 < (int)nf) ? q.off[t + 1] : mf;
        if (ot < e0 || ot >= e1 || endt <= e1) continue;  // not the head of a split list
        double acc = gs.plast[c];
        for (uint32_t c2 = c + 1; c2 < nchunks && q.part[c2] == t; ++c2) acc += gs.pfirst[c2];
        fin(q.v[t], acc);
    }
}

// Visit every edge (v_i -> u) of the queue once, load-balanced over edges:
// op(u, v_i) runs on one lane per edge.  Used where the per-edge work has no
// reduction (connected-component hooking).
template <int CH, class Op>
__global__ __launch_bounds__(GFR_BLOCK) void for_each_edge(FrontierQ q, const uint32_t *nf_p,
                                                           const uint32_t *mf_p, const int32_t *C,
                                                           Op op)
{
    const uint32_t nf = *nf_p, mf = *mf_p;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t e0 = c * CH;
        const uint32_t e1 = min(e0 + (uint32_t)CH, mf);
        const int s = q.part[c];
        const int t = (c + 1 < nchunks) ? q.part[c + 1] : (int)nf - 1;
        const int cnt = t - s + 1;
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            s_off[i] = q.off[s + i];
            s_row[i] = q.row[s + i];
            s_v[i] = q.v[s + i];
        }
        __syncthreads();
        for (uint32_t k = 0; k < (uint32_t)CH; k += GFR_BLOCK) {
            const uint32_t e = e0 + k + threadIdx.x;
            const bool valid = e < e1;
            int32_t u = 0, v = 0;
            if (valid) {
                const int i = upper_index(s_off, 0, cnt - 1, e);
                u = C[s_row[i] + (int32_t)(e - s_off[i])];
                v = s_v[i];
            }
            op(valid, u, v);   // called by every lane (converged), valid marks real edges
        }
    }
}

}  // namespace gfr
