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
#include "compact.h"
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

// byte[list[i]] = 1 for i < k
__global__ void set_bytes(const int32_t *list, int32_t k, uint8_t *byte)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) byte[list[i]] = 1;
}

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

// ---------------------------------------------------------------------------
// PageRank with per-vertex convergence filtering (Sec. 5.5, the paper's own
// formulation): the frontier starts with every vertex; an iteration
// recomputes the rank of the frontier's vertices from the ranks of the
// previous iterate (vertices outside keep their last value), then the filter
// keeps only the vertices whose rank moved by at least vertex_tol.  The
// decision is taken in FP64, so ranks and contributions are FP64 here.
//
// Vertices with edges live in a FrontierQ rebuilt every iteration by the
// ordered compaction from one persistent byte per vertex (1 = in the
// frontier); that byte array is also the final frontier membership.
// Vertices without edges all share one value at every step (same start, same
// update), so they are carried as a single class in the control block.
//
// Per iteration (every launch checks `done`):
//   gather_chunks / gather_fixup   S(v) over the frontier queue
//   pf_finalize                    x'(v) = (1-d)/N + d (S(v) + D/N), change,
//                                  contribution, keep byte, L1 partials
//   compact_kernel<PfMarks>        next queue; the last work-group updates the
//                                  zero-degree class, D, the iteration count
//                                  and `done`

struct PfCtl {
    uint32_t done;       // first word: read back by the host
    uint32_t iters;
    uint32_t max_iter;
    uint32_t parity;     // compaction status buffer in use
    uint32_t nf, mf;     // current queue: entries and edges
    uint32_t iso_active; // the zero-degree class is in the frontier
    uint32_t err;        // compaction look-back error
    double n_iso;        // number of zero-degree vertices
    double x_iso;        // their common rank
    double D;            // rank held by zero-degree vertices
    double l1;           // summed change of the last iteration
    double tol;
    double damping;
    double updates;      // vertex updates over all iterations
    double edges;        // neighbour-list entries gathered over all iterations
};

struct PfOp {
    const double *contrib;
    __device__ double operator()(int32_t u, int32_t) const { return contrib[u]; }
};

__global__ __launch_bounds__(GFR_BLOCK) void pf_init(const int32_t *R, int32_t n, double *x, double *contrib,
                                                      uint8_t *keep)
{
    const double xv = 1.0 / (double)n;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const int32_t deg = R[v + 1] - R[v];
        x[v] = xv;
        contrib[v] = deg > 0 ? xv / (double)deg : 0.0;
        keep[v] = deg > 0 ? 1 : 0;
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void pf_finalize(const int32_t *R, int32_t n, FrontierQ q, double *x,
                                                          double *contrib, const double *sum, uint8_t *keep,
                                                          double *part, const PfCtl *ctl)
{
    if (ctl->done) return;
    const uint32_t nf = ctl->nf;
    const double d = ctl->damping, N = (double)n, tol = ctl->tol;
    const double tele = (1.0 - d) / N, dn = ctl->D / N;
    double l1 = 0.0, zero = 0.0;
    for (uint32_t i = blockIdx.x * GFR_BLOCK + threadIdx.x; i < nf; i += gridDim.x * GFR_BLOCK) {
        const int32_t v = q.v[i];
        const double y = tele + d * (sum[v] + dn);
        const double dx = fabs(y - x[v]);
        l1 += dx;
        x[v] = y;
        contrib[v] = y / (double)(R[v + 1] - R[v]);
        keep[v] = dx >= tol ? 1 : 0;
    }
    block_sum2(l1, zero);
    if (threadIdx.x == 0) part[blockIdx.x] = l1;
}

struct PfMarks {
    const uint8_t *keep;
    const double *part;   // L1 partials of pf_finalize
    uint32_t nparts;
    PfCtl *ctl;
    int32_t n;
    uint32_t first;       // the launch that builds the initial queue

    __device__ bool skip() const { return !first && ctl->done; }
    __device__ uint32_t mask(uint32_t w) const { return marks_to_mask(keep + 32ull * w); }
    __device__ void partial(uint32_t) {}
    __device__ void control(uint32_t nf2, uint32_t mf2) const
    {
        double l1 = 0.0, zero = 0.0;
        if (!first)
            for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) l1 += part[i];
        block_sum2(l1, zero);
        if (threadIdx.x != 0) return;
        PfCtl *c = ctl;
        const double N = (double)n;
        if (first) {
            c->n_iso = (double)(n - (int32_t)nf2);
            c->x_iso = 1.0 / N;
            c->iso_active = nf2 < (uint32_t)n ? 1u : 0u;
            c->D = c->n_iso * c->x_iso;
            c->iters = 0;
            c->l1 = 0.0;
            c->updates = 0.0;
            c->edges = 0.0;
            c->done = (nf2 == 0 && !c->iso_active) || c->max_iter == 0 ? 1u : 0u;
        } else {
            c->updates += (double)c->nf;
            c->edges += (double)c->mf;
            if (c->iso_active) {
                const double d = c->damping;
                const double y = (1.0 - d) / N + d * (0.0 + c->D / N);
                const double dx = fabs(y - c->x_iso);
                l1 += c->n_iso * dx;
                c->x_iso = y;
                c->iso_active = dx >= c->tol ? 1u : 0u;
                c->updates += c->n_iso;
            }
            c->D = c->n_iso * c->x_iso;
            c->l1 = l1;
            c->iters += 1;
            c->done = (nf2 == 0 && !c->iso_active) || c->iters >= c->max_iter ? 1u : 0u;
        }
        c->nf = nf2;
        c->mf = mf2;
        c->parity ^= 1u;
    }
};

__global__ __launch_bounds__(GFR_BLOCK) void pf_output(const int32_t *R, int32_t n, const double *x,
                                                        const uint8_t *keep, const PfCtl *ctl, double *rank,
                                                        uint8_t *active)
{
    const double xi = ctl->x_iso;
    const uint8_t ai = ctl->iso_active ? 1 : 0;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const bool iso = R[v + 1] == R[v];
        rank[v] = iso ? xi : x[v];
        active[v] = iso ? ai : keep[v];
    }
}

const uint8_t *run_pagerank_filtered(Ctx &c, Graph &g, double damping, double vertex_tol, int32_t max_iter,
                                     double *rank, int32_t *iters, double *l1, hipStream_t s)
{
    const int32_t n = g.n;
    const int G = grid_blocks(c, 4);
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    const size_t nch = (size_t)(g.m / GATHER_CH) + 2;
    c.arena.reserve(3 * al256(8ull * n) + al256(32ull * nwords) + al256(n) + 3 * al256(4ull * n) +
                    al256(4 * nch) + 2 * al256(8 * nch) + al256(8ull * G) + al256(16ull * cg.blocks) +
                    al256(sizeof(PfCtl)));
    double *x = c.arena.take<double>(n);
    double *contrib = c.arena.take<double>(n);
    double *sum = c.arena.take<double>(n);
    uint8_t *keep = c.arena.take<uint8_t>(32ull * nwords);
    uint8_t *active = c.arena.take<uint8_t>(n);
    FrontierQ q{c.arena.take<int32_t>(n), c.arena.take<uint32_t>(n), c.arena.take<int32_t>(n),
                c.arena.take<int32_t>(nch)};
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    double *part = c.arena.take<double>(G);
    unsigned long long *status = c.arena.take<unsigned long long>(2ull * cg.blocks);
    PfCtl *ctl = c.arena.take<PfCtl>(1);

    PfCtl h{};
    h.max_iter = (uint32_t)max_iter;
    h.tol = vertex_tol;
    h.damping = damping;
    GFR_HIP(hipMemcpyAsync(ctl, &h, sizeof h, hipMemcpyHostToDevice, s));
    fill_u32(keep, 0u, 8ull * nwords, s);
    fill_u32(status, 0u, 4ull * cg.blocks, s);
    const int32_t *R = g.R.as<int32_t>(), *C = g.C.as<int32_t>();
    hipLaunchKernelGGL(pf_init, dim3(G), dim3(GFR_BLOCK), 0, s, R, n, x, contrib, keep);
    PfMarks mk{keep, part, (uint32_t)G, ctl, n, 1u};
    hipLaunchKernelGGL(compact_kernel<PfMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, R, n, nwords, cg.wpt, mk, q,
                       (uint32_t)GATHER_CH, status, &ctl->parity, &ctl->err);
    GFR_LAUNCH_CHECK();
    mk.first = 0u;

    PfOp op{contrib};
    PrFin fin{sum};
    auto launch = [&]() {
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, PfOp, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, q, &ctl->nf,
                           &ctl->mf, C, op, fin, gs, &ctl->done);
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, q, &ctl->nf,
                           &ctl->mf, fin, gs, &ctl->done);
        hipLaunchKernelGGL(pf_finalize, dim3(G), dim3(GFR_BLOCK), 0, s, R, n, q, x, contrib, sum, keep, part, ctl);
        hipLaunchKernelGGL(compact_kernel<PfMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, R, n, nwords, cg.wpt, mk,
                           q, (uint32_t)GATHER_CH, status, &ctl->parity, &ctl->err);
    };
    const int32_t first = max_iter < 8 ? max_iter : 8;
    run_until_done(c, &ctl->done, 1u, first, (int64_t)max_iter + 8, s, launch);
    hipLaunchKernelGGL(pf_output, dim3(G), dim3(GFR_BLOCK), 0, s, R, n, x, keep, ctl, rank, active);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    if (h.err) fail(GFR_E_DEVICE, "pagerank_filtered: frontier compaction look-back timed out");
    *iters = (int32_t)h.iters;
    *l1 = h.l1;
    c.stats.v["iterations"] = h.iters;
    c.stats.v["l1"] = h.l1;
    c.stats.v["vertex_updates"] = h.updates;
    c.stats.v["edges_gathered"] = h.edges;
    c.stats.v["final_frontier"] = (double)h.nf + (h.iso_active ? h.n_iso : 0.0);
    return active;
}

// ---------------------------------------------------------------------------
// Personalized PageRank: the teleport vector p is uniform over a seed set and
// also receives the rank of zero-degree vertices,
//   x_0 = p,  x_{k+1}(v) = (1-d) p(v) + d (S(v) + D_k p(v)),
// the ranking that seeds the bipartite who-to-follow pipeline.  Same launch
// structure as run_pagerank (full-queue gather, finalize, one-group reduce,
// speculative iterations), with FP64 ranks and contributions.

struct PpOp {
    const double *contrib;
    __device__ double operator()(int32_t u, int32_t) const { return contrib[u]; }
};

__global__ __launch_bounds__(GFR_BLOCK) void ppr_init(const int32_t *R, int32_t n, const uint8_t *seed, double invk,
                                                       double *x0, double *contrib, double *part)
{
    double dang = 0.0, zero = 0.0;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const int32_t deg = R[v + 1] - R[v];
        const double xv = seed[v] ? invk : 0.0;
        x0[v] = xv;
        if (deg > 0) contrib[v] = xv / (double)deg;
        else dang += xv;
    }
    block_sum2(dang, zero);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 0.0;
        part[2 * blockIdx.x + 1] = dang;
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void ppr_finalize(const int32_t *R, int32_t n, const uint8_t *seed,
                                                           double invk, double *xa, double *xb, double *contrib,
                                                           const double *sum, double *part, PrCtl *ctl)
{
    if (ctl->done) return;
    const uint32_t k = ctl->iters;
    const double *xo = (k & 1) ? xb : xa;
    double *xn = (k & 1) ? xa : xb;
    const double d = ctl->damping, D = ctl->D;
    double l1 = 0.0, dang = 0.0;
    for (int32_t v = blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += gridDim.x * GFR_BLOCK) {
        const int32_t deg = R[v + 1] - R[v];
        const double s = deg > 0 ? sum[v] : 0.0;
        const double p = seed[v] ? invk : 0.0;
        const double x = (1.0 - d) * p + d * (s + D * p);
        l1 += fabs(x - xo[v]);
        xn[v] = x;
        if (deg > 0) contrib[v] = x / (double)deg;
        else dang += x;
    }
    block_sum2(l1, dang);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = l1;
        part[2 * blockIdx.x + 1] = dang;
    }
}

void run_ppr(Ctx &c, Graph &g, const int32_t *seeds, int32_t k, double damping, double tol, int32_t max_iter,
             double *rank, int32_t *iters, double *l1, hipStream_t s)
{
    const int32_t n = g.n;
    const int G = grid_blocks(c, 4);
    const size_t nch = (size_t)(g.m + GATHER_CH - 1) / GATHER_CH + 1;
    c.arena.reserve(4 * al256(8ull * n) + al256(4ull * ((n + 3) / 4)) + al256(4ull * k) + 2 * al256(8 * nch) +
                    al256(16ull * G) + al256(sizeof(PrCtl)));
    double *xa = c.arena.take<double>(n);
    double *xb = c.arena.take<double>(n);
    double *contrib = c.arena.take<double>(n);
    double *sum = c.arena.take<double>(n);
    uint8_t *seed = c.arena.take<uint8_t>(4ull * ((n + 3) / 4));
    int32_t *dseeds = c.arena.take<int32_t>(k);
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    double *part = c.arena.take<double>(2 * (size_t)G);
    PrCtl *ctl = c.arena.take<PrCtl>(1);
    const double invk = 1.0 / (double)k;

    PrCtl h{};
    h.max_iter = (uint32_t)max_iter;
    h.tol = tol;
    h.damping = damping;
    GFR_HIP(hipMemcpyAsync(ctl, &h, sizeof h, hipMemcpyHostToDevice, s));
    GFR_HIP(hipMemcpyAsync(dseeds, seeds, 4ull * k, hipMemcpyHostToDevice, s));
    fill_u32(seed, 0u, (n + 3) / 4, s);
    hipLaunchKernelGGL(set_bytes, dim3((k + GFR_BLOCK - 1) / GFR_BLOCK), dim3(GFR_BLOCK), 0, s, dseeds, k, seed);
    hipLaunchKernelGGL(ppr_init, dim3(G), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(), n, seed, invk, xa, contrib, part);
    hipLaunchKernelGGL(pr_reduce, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, ctl, 1u);
    GFR_LAUNCH_CHECK();

    PpOp op{contrib};
    PrFin fin{sum};
    const int32_t *C = g.C.as<int32_t>();
    auto launch = [&]() {
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, PpOp, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full,
                           g.full_counts, g.full_counts + 1, C, op, fin, gs, &ctl->done);
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, PrFin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full,
                           g.full_counts, g.full_counts + 1, fin, gs, &ctl->done);
        hipLaunchKernelGGL(ppr_finalize, dim3(G), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(), n, seed, invk, xa, xb,
                           contrib, sum, part, ctl);
        hipLaunchKernelGGL(pr_reduce, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, ctl, 0u);
    };
    const int32_t first = max_iter < 8 ? max_iter : 8;
    run_until_done(c, &ctl->done, 1u, first, (int64_t)max_iter + 8, s, launch);
    GFR_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    const double *xf = (h.iters & 1) ? xb : xa;
    GFR_HIP(hipMemcpyAsync(rank, xf, 8ull * n, hipMemcpyDeviceToDevice, s));
    *iters = (int32_t)h.iters;
    *l1 = h.l1;
    c.stats.v["iterations"] = h.iters;
    c.stats.v["l1"] = h.l1;
}

}  // namespace gfr
