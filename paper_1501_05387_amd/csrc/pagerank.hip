// pagerank.hip -- PageRank by power iteration over the full vertex frontier
// (Sec. 5.5: the frontier holds every vertex, so an iteration is a sparse
// matrix-vector product).  Pull formulation: each vertex gathers its
// neighbours' contributions x(u)/deg(u), so no floating-point atomics are
// needed and every sum has a fixed order.  Ranks and contributions are stored
// in FP32; per-vertex sums, the dangling mass and the L1 change are FP64.
//
// Per iteration (all launches check a device `done` word, so iterations are
// enqueued speculatively):
//   gather_chunks / gather_fixup   S(v) = sum over u in N(v) of contrib(u)
//   pr_finalize                    x'(v) = (1-d)/N + d (S(v) + D/N), L1, next
//                                  contributions and dangling mass D
#include "engine.h"
#include "gather.h"

namespace gfr {

struct PrCtl {
    uint32_t done;      // first word: read back by the host
    uint32_t iters;
    uint32_t max_iter;
    uint32_t pad;
    double D;           // rank held by zero-degree vertices, current iterate
    double l1;          // L1 change of the last iteration
    double tol;
    double damping;
};

struct PrOp {
    const float *contrib;
    __device__ double operator()(int32_t u, int32_t) const { return (double)contrib[u]; }
};

struct PrFin {
    double *sum;
    __device__ void operator()(int32_t v, double s) const { sum[v] = s; }
};

// Fixed-order block reduction of two FP64 values (wave butterfly, then the
// four wave results in wave order).
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double sa[GFR_WAVES], sb[GFR_WAVES];
    a = wave_sum_f64(a);
    b = wave_sum_f64(b);
    const int w = threadIdx.x / 64;
    __syncthreads();
    if (lane_id() == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int i = 0; i < GFR_WAVES; ++i) {
            x += sa[i];
            y += sb[i];
        }
        a = x;
        b = y;
    }
}

// iteration 0: x = 1/N, contributions, dangling mass
__global__ __launch_bounds__(GFR_BLOCK) void pr_init(const int32_t *R, int32_t n, float *x0, float *contrib,
                                                      double *part, PrCtl *ctl)
{
    const float xv = (float)(1.0 / (double)n);
    double dang = 0.0, zero = 0.0;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const int32_t deg = R[v + 1] - R[v];
        x0[v] = xv;
        if (deg > 0) contrib[v] = xv / (float)deg;
        else dang += (double)xv;
    }
    block_sum2(dang, zero);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 0.0;
        part[2 * blockIdx.x + 1] = dang;
    }
}

// One work-group: reduce the per-group partials of pr_init / pr_finalize in a
// fixed order and run the iteration control.  first != 0: after pr_init.
__global__ __launch_bounds__(GFR_BLOCK) void pr_reduce(const double *part, uint32_t nparts, PrCtl *ctl,
                                                       uint32_t first)
{
    if (!first && ctl->done) return;
    double l1 = 0.0, dang = 0.0;
    for (uint32_t b = threadIdx.x; b < nparts; b += GFR_BLOCK) {
        l1 += part[2 * b];
        dang += part[2 * b + 1];
    }
    block_sum2(l1, dang);
    if (threadIdx.x == 0) {
        ctl->D = dang;
        if (first) {
            ctl->iters = 0;
            ctl->l1 = 0.0;
            ctl->done = 0;
        } else {
            const uint32_t k = ctl->iters + 1;
            ctl->iters = k;
            ctl->l1 = l1;
            if ((ctl->tol > 0.0 && l1 < ctl->tol) || k >= ctl->max_iter) ctl->done = 1;
        }
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void pr_finalize(const int32_t *R, int32_t n, float *xa, float *xb,
                                                          float *contrib, const double *sum,
                                                          double *part, PrCtl *ctl)
{
    if (ctl->done) return;
    const uint32_t k = ctl->iters;
    const float *xo = (k & 1) ? xb : xa;
    float *xn = (k & 1) ? xa : xb;
    const double d = ctl->damping, N = (double)n;
    const double base = (1.0 - d) / N + d * ctl->D / N;
    double l1 = 0.0, dang = 0.0;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const int32_t deg = R[v + 1] - R[v];
        const double s = deg > 0 ? sum[v] : 0.0;
        const float x = (float)(base + d * s);
        l1 += fabs((double)x - (double)xo[v]);
        xn[v] = x;
        if (deg > 0) contrib[v] = x / (float)deg;
        else dang += (double)x;
    }
    block_sum2(l1, dang);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = l1;
        part[2 * blockIdx.x + 1] = dang;
    }
}

void run_pagerank(Ctx &c, Graph &g, float damping, double tol, int32_t max_iter, float *rank,
                  int32_t *iters, double *l1, hipStream_t s)
{
    const int32_t n = g.n;
    const int G = grid_blocks(c, 4);
    const size_t nch = (size_t)(g.m + GATHER_CH - 1) / GATHER_CH + 1;
    c.arena.reserve(3 * al256(4ull * n) + al256(8ull * n) + 2 * al256(8 * nch) + al256(16ull * G) +
                    al256(sizeof(PrCtl)));
    float *xa = c.arena.take<float>(n);
    float *xb = c.arena.take<float>(n);
    float *contrib = c.arena.take<float>(n);
    double *sum = c.arena.take<double>(n);
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    double *part = c.arena.take<double>(2 * (size_t)G);
    PrCtl *ctl = c.arena.take<PrCtl>(1);

    PrCtl h{};
    h.max_iter = (uint32_t)max_iter;
    h.tol = tol;
    h.damping = damping;
    GFR_HIP(hipMemcpyAsync(ctl, &h, sizeof h, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(pr_init, dim3(G), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(), n, xa, contrib, part, ctl);
    hipLaunchKernelGGL(pr_reduce, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, ctl, 1u);
    GFR_LAUNCH_CHECK();

    PrOp op{contrib};
    PrFin fin{sum};
    const int32_t *C = g.C.as<int32_t>();
    auto launch = [&]() {
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, PrOp, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full,
                           g.full_counts, g.full_counts + 1, C, op, fin, gs, &ctl->done);
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full,
                           g.full_counts, g.full_counts + 1, fin, gs, &ctl->done);
        hipLaunchKernelGGL(pr_finalize, dim3(G), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(), n, xa, xb, contrib,
                           sum, part, ctl);
        hipLaunchKernelGGL(pr_reduce, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, ctl, 0u);
    };
    const int32_t first = max_iter < 8 ? max_iter : 8;
    run_until_done(c, &ctl->done, 1u, first, (int64_t)max_iter + 8, s, launch);
    GFR_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    const float *xf = (h.iters & 1) ? xb : xa;
    GFR_HIP(hipMemcpyAsync(rank, xf, 4ull * n, hipMemcpyDeviceToDevice, s));
    *iters = (int32_t)h.iters;
    *l1 = h.l1;
    c.stats.v["iterations"] = h.iters;
    c.stats.v["l1"] = h.l1;
}

}  // namespace gfr
