// rank.hip -- the 2-hop advance and the bipartite node rankings (SALSA, HITS)
// built from the same operators (Sec. 4.1 lists pulling values from vertices
// two hops away through an edge frontier as a use of advance; Sec. 5.5 names
// personalized PageRank, SALSA and HITS on bipartite graphs as rankings
// written with it).
//
// 2-hop walk counts, count(v) = number of walks s - u - v from a seed set:
//   1. the seeds become a frontier queue (mark bytes + ordered compaction);
//   2. advance over the seeds' edges: c1(u) += 1 per seed neighbour (integer
//      atomics), marking u;
//   3. the marked vertices become the middle frontier (compaction);
//   4. push: advance over the middle frontier's edges, count(v) += c1(u)
//      (64-bit atomics, ~13 G/s on MI355X); or pull, when the middle
//      frontier holds more than m / alpha edges (default alpha 10: a pull
//      sweep of all m edges runs near 125 G edges/s): every vertex gathers
//      the sum of c1 over its list with the segmented FP64 gather, exact
//      because every partial sum is an integer below 2^53.
//
// SALSA / HITS on a bipartite graph (hubs [0, nl), authorities [nl, n)):
// each side is a frontier queue built once; an iteration is a gather over
// the authorities' lists (of hub values) followed by a gather over the hubs'
// lists (of the new authority values).  SALSA divides every value by its
// vertex's degree (a random walk); HITS scales each side to unit L2 norm
// after its gather, the norm being reduced in a fixed order.
#include "compact.h"
#include "engine.h"
#include "gather.h"

namespace gfr {

// ------------------------------------------------------------ frontiers

// the vertices marked in a byte array (marks consumed)
struct ByteMarks {
    uint8_t *mark;
    unsigned long long *out;   // (entries << 32) | edges of the new queue
    uint32_t *parity;
    __device__ bool skip() const { return false; }
    __device__ uint32_t mask(uint32_t w) const
    {
        const uint32_t m = marks_to_mask(mark + 32ull * w);
        if (m) clear_marks(mark + 32ull * w);
        return m;
    }
    __device__ void partial(uint32_t) {}
    __device__ void control(uint32_t nf, uint32_t mf) const
    {
        if (threadIdx.x == 0) {
            *out = ((unsigned long long)nf << 32) | mf;
            *parity ^= 1u;
        }
    }
};

// the vertices of [lo, hi)
struct RangeMarks {
    int32_t lo, hi;
    unsigned long long *out;
    uint32_t *parity;
    __device__ bool skip() const { return false; }
    __device__ uint32_t mask(uint32_t w) const
    {
        const int64_t v0 = 32ll * w;
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 32; ++i) m |= (v0 + i >= lo && v0 + i < hi) ? 1u << i : 0u;
        return m;
    }
    __device__ void partial(uint32_t) {}
    __device__ void control(uint32_t nf, uint32_t mf) const
    {
        if (threadIdx.x == 0) {
            *out = ((unsigned long long)nf << 32) | mf;
            *parity ^= 1u;
        }
    }
};

__global__ void mark_list(const int32_t *list, int32_t k, uint8_t *mark)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) mark[list[i]] = 1;
}

// Scratch for building queues with the ordered compaction.
struct QueueBuilder {
    uint32_t nwords;
    CompactGeom cg;
    unsigned long long *status;
    uint32_t *cw;   // [0] parity, [1] look-back error
    static size_t bytes(int32_t n, int num_cu)
    {
        const uint32_t nw = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
        return al256(16ull * compact_geom(nw, num_cu).blocks) + al256(256);
    }
    void init(Ctx &c, int32_t n, hipStream_t s)
    {
        nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
        cg = compact_geom(nwords, c.num_cu);
        status = c.arena.take<unsigned long long>(2ull * cg.blocks);
        cw = c.arena.take<uint32_t>(64);
        fill_u32(status, 0u, 4ull * cg.blocks, s);
        fill_u32(cw, 0u, 64, s);
    }
    template <class M> void build(const Graph &g, M mk, FrontierQ q, hipStream_t s)
    {
        hipLaunchKernelGGL(compact_kernel<M>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(), g.n, nwords,
                           cg.wpt, mk, q, (uint32_t)GATHER_CH, status, cw, cw + 1);
        GFR_LAUNCH_CHECK();
    }
    void check(Ctx &c, hipStream_t s, const char *who)
    {
        GFR_HIP(hipMemcpyAsync(c.pinned, cw + 1, 4, hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        if (c.pinned[0]) fail(GFR_E_DEVICE, std::string(who) + ": frontier compaction look-back timed out");
    }
};

static FrontierQ take_queue(Ctx &c, const Graph &g)
{
    const size_t nparts = (size_t)(g.m / GATHER_CH) + 2;
    return FrontierQ{c.arena.take<int32_t>(g.n), c.arena.take<uint32_t>(g.n), c.arena.take<int32_t>(g.n),
                     c.arena.take<int32_t>(nparts)};
}

static size_t queue_bytes(const Graph &g)
{
    return 3 * al256(4ull * g.n) + al256(4ull * ((size_t)(g.m / GATHER_CH) + 2));
}

// ---------------------------------------------------------------- 2-hop

struct Hop1Op {
    uint32_t *c1;
    uint8_t *mark;
    __device__ void operator()(bool valid, int32_t u, int32_t) const
    {
        if (valid) {
            atomicAdd(c1 + u, 1u);
            mark[u] = 1;
        }
    }
};

struct Hop2PushOp {
    const uint32_t *c1;
    unsigned long long *count;
    __device__ void operator()(bool valid, int32_t v, int32_t u) const
    {
        if (valid) atomicAdd(count + v, (unsigned long long)c1[u]);
    }
};

struct Hop2PullOp {
    const uint32_t *c1;
    __device__ double operator()(int32_t u, int32_t) const { return (double)c1[u]; }
};

struct Hop2Fin {
    unsigned long long *count;
    __device__ void operator()(int32_t v, double s) const { count[v] = (unsigned long long)s; }
};

void run_two_hop(Ctx &c, Graph &g, const int32_t *seeds, int32_t k, uint64_t *count, hipStream_t s)
{
    const int32_t n = g.n;
    const int G = grid_blocks(c, 4);
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nch = (size_t)(g.m / GATHER_CH) + 2;
    c.arena.reserve(al256(4ull * n) + al256(32ull * nwords) + queue_bytes(g) + al256(4ull * k) + al256(16) +
                    2 * al256(8 * nch) + QueueBuilder::bytes(n, c.num_cu));
    uint32_t *c1 = c.arena.take<uint32_t>(n);
    uint8_t *mark = c.arena.take<uint8_t>(32ull * nwords);
    FrontierQ q = take_queue(c, g);
    int32_t *dseeds = c.arena.take<int32_t>(k);
    unsigned long long *ctr = c.arena.take<unsigned long long>(2);
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    QueueBuilder qb;
    qb.init(c, n, s);
    fill_u32(c1, 0u, n, s);
    fill_u32(mark, 0u, 8ull * nwords, s);
    fill_u32(count, 0u, 2ull * n, s);
    GFR_HIP(hipMemcpyAsync(dseeds, seeds, 4ull * k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mark_list, dim3((k + GFR_BLOCK - 1) / GFR_BLOCK), dim3(GFR_BLOCK), 0, s, dseeds, k, mark);
    qb.build(g, ByteMarks{mark, ctr, qb.cw}, q, s);
    const uint32_t *q1 = (const uint32_t *)ctr;   // [0] edges, [1] entries
    const int32_t *C = g.C.as<int32_t>();
    hipLaunchKernelGGL((for_each_edge<GATHER_CH, Hop1Op>), dim3(G), dim3(GFR_BLOCK), 0, s, q, q1 + 1, q1, C,
                       Hop1Op{c1, mark});
    qb.build(g, ByteMarks{mark, ctr + 1, qb.cw}, q, s);
    GFR_HIP(hipMemcpyAsync(c.pinned, ctr, 16, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    const uint32_t mf1 = c.pinned[0], mf2 = c.pinned[2];
    const int force = c.opt.twohop_direction;
    const bool pull = force == 2 || (force == 0 && (double)mf2 > (double)g.m / c.opt.twohop_alpha);
    unsigned long long *cnt = (unsigned long long *)count;
    if (pull) {
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, Hop2PullOp, Hop2Fin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full,
                           g.full_counts, g.full_counts + 1, C, Hop2PullOp{c1}, Hop2Fin{cnt}, gs,
                           c.zero_word.as<uint32_t>());
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, Hop2Fin>), dim3(G), dim3(GFR_BLOCK), 0, s, g.full, g.full_counts,
                           g.full_counts + 1, Hop2Fin{cnt}, gs, c.zero_word.as<uint32_t>());
    } else {
        const uint32_t *q2 = (const uint32_t *)(ctr + 1);
        hipLaunchKernelGGL((for_each_edge<GATHER_CH, Hop2PushOp>), dim3(G), dim3(GFR_BLOCK), 0, s, q, q2 + 1, q2, C,
                           Hop2PushOp{c1, cnt});
    }
    GFR_LAUNCH_CHECK();
    qb.check(c, s, "two_hop");
    c.stats.v["pull_levels"] = pull ? 1.0 : 0.0;
    c.stats.v["edges_inspected"] = (double)mf1 + (pull ? (double)g.m : (double)mf2);
    c.stats.v["middle_vertices"] = (double)c.pinned[3];
}

// ------------------------------------------------------- SALSA and HITS

// one side's values, read by the other side's gather: SALSA x/deg, HITS x*scale
struct SideOp {
    const double *x;
    const double *scale;   // HITS: 1/||x||_2 of the side (device scalar), SALSA: null
    __device__ double operator()(int32_t u, int32_t) const
    {
        const double v = x[u];
        return scale ? v * *scale : v;
    }
};

// SALSA: stores x(v) / deg(v); HITS: stores the unscaled sum
struct SideFin {
    const int32_t *R;
    double *x;
    bool walk;
    __device__ void operator()(int32_t v, double s) const { x[v] = walk ? s / (double)(R[v + 1] - R[v]) : s; }
};

// per-group sums of squares over a queue, in a fixed order
__global__ __launch_bounds__(GFR_BLOCK) void side_sumsq(FrontierQ q, const uint32_t *nf_p, const double *x,
                                                         double *part)
{
    const uint32_t nf = *nf_p;
    double a = 0.0;
    for (uint32_t i = blockIdx.x * GFR_BLOCK + threadIdx.x; i < nf; i += gridDim.x * GFR_BLOCK) {
        const double v = x[q.v[i]];
        a += v * v;
    }
    __shared__ double sw[GFR_WAVES];
    a = wave_sum_f64(a);
    if (lane_id() == 0) sw[threadIdx.x / 64] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < GFR_WAVES; ++i) t += sw[i];
        part[blockIdx.x] = t;
    }
}

// 1/sqrt of the summed partials (1 for a zero vector, which stays zero)
__global__ __launch_bounds__(GFR_BLOCK) void side_inv_norm(const double *part, uint32_t nparts, double *inv)
{
    double a = 0.0;
    for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) a += part[i];
    __shared__ double sw[GFR_WAVES];
    a = wave_sum_f64(a);
    if (lane_id() == 0) sw[threadIdx.x / 64] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < GFR_WAVES; ++i) t += sw[i];
        *inv = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
    }
}

// hub values at the start (every hub, isolated ones included)
__global__ void hub_start(double *x, int32_t nl, const int32_t *R, double h0, bool walk)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nl; v += gridDim.x * blockDim.x) {
        const int32_t deg = R[v + 1] - R[v];
        x[v] = walk ? (deg > 0 ? h0 / (double)deg : 0.0) : h0;
    }
}

// final scores: SALSA x*deg, HITS x*scale; a vertex without edges scores 0
// once an iteration has run (the start value h0 before)
__global__ void side_output(const double *x, int32_t lo, int32_t hi, const int32_t *R, bool walk, const double *scale,
                            int32_t iters, double h0, double *out)
{
    for (int32_t v = lo + blockIdx.x * blockDim.x + threadIdx.x; v < hi; v += gridDim.x * blockDim.x) {
        const int32_t deg = R[v + 1] - R[v];
        double r;
        if (iters == 0) r = h0;
        else if (deg == 0) r = 0.0;
        else r = walk ? x[v] * (double)deg : x[v] * *scale;
        out[v - lo] = r;
    }
}

__global__ void count_same_side_edges(const int32_t *R, const int32_t *C, int32_t n, int32_t nl, uint32_t *bad)
{
    uint32_t b = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        for (int32_t e = R[v]; e < R[v + 1]; ++e) b += ((v < nl) == (C[e] < nl)) ? 1u : 0u;
    if (b) atomicAdd(bad, b);
}

void check_bipartite(Ctx &c, Graph &g, int32_t nl, hipStream_t s)
{
    if (g.bip_checked_nl == nl) return;
    uint32_t *bad = c.arena.take<uint32_t>(1);
    fill_u32(bad, 0u, 1, s);
    hipLaunchKernelGGL(count_same_side_edges, dim3(grid_blocks(c, 4)), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(),
                       g.C.as<int32_t>(), g.n, nl, bad);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, bad, 4, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    if (c.pinned[0]) fail(GFR_E_INVALID, "bipartite ranking: an edge joins two vertices of the same side");
    g.bip_checked_nl = nl;
}

void run_bipartite_rank(Ctx &c, Graph &g, int32_t nl, int32_t iters, bool walk, double *hub, double *auth,
                        hipStream_t s)
{
    const int32_t n = g.n;
    const int G = grid_blocks(c, 4);
    const size_t nch = (size_t)(g.m / GATHER_CH) + 2;
    c.arena.reserve(al256(8ull * n) + 2 * queue_bytes(g) + 2 * al256(8 * nch) + al256(8ull * G) + al256(64) +
                    al256(16) + al256(4) + QueueBuilder::bytes(n, c.num_cu) + 2 * al256(8ull * n));
    check_bipartite(c, g, nl, s);
    double *x = c.arena.take<double>(n);   // hubs [0, nl), authorities [nl, n)
    FrontierQ qh = take_queue(c, g), qa = take_queue(c, g);
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    double *part = c.arena.take<double>(G);
    double *inv = c.arena.take<double>(8);   // [0] hubs, [1] authorities
    unsigned long long *ctr = c.arena.take<unsigned long long>(2);
    double *hub_dev = c.arena.take<double>(n);
    double *auth_dev = hub_dev + nl;
    QueueBuilder qb;
    qb.init(c, n, s);
    qb.build(g, RangeMarks{0, nl, ctr, qb.cw}, qh, s);
    qb.build(g, RangeMarks{nl, n, ctr + 1, qb.cw}, qa, s);
    const uint32_t *ch = (const uint32_t *)ctr, *ca = (const uint32_t *)(ctr + 1);
    const double h0 = walk ? 1.0 / (double)nl : 1.0 / sqrt((double)nl);
    hipLaunchKernelGGL(hub_start, dim3(G), dim3(GFR_BLOCK), 0, s, x, nl, g.R.as<int32_t>(), h0, walk);
    fill_u32(inv, 0u, 16, s);
    {
        const double one[2] = {1.0, 1.0};
        GFR_HIP(hipMemcpyAsync(inv, one, sizeof one, hipMemcpyHostToDevice, s));
    }
    const int32_t *R = g.R.as<int32_t>(), *C = g.C.as<int32_t>();
    const uint32_t *never = c.zero_word.as<uint32_t>();
    for (int32_t it = 0; it < iters; ++it) {
        // authorities gather the hubs' values, then hubs gather the new authority values
        SideOp opa{x, walk ? nullptr : inv + 0};
        SideFin fin{R, x, walk};
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, SideOp, SideFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qa, ca + 1, ca,
                           C, opa, fin, gs, never);
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, SideFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qa, ca + 1, ca, fin, gs,
                           never);
        if (!walk) {
            hipLaunchKernelGGL(side_sumsq, dim3(G), dim3(GFR_BLOCK), 0, s, qa, ca + 1, x, part);
            hipLaunchKernelGGL(side_inv_norm, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, inv + 1);
        }
        SideOp oph{x, walk ? nullptr : inv + 1};
        hipLaunchKernelGGL((gather_chunks<GATHER_CH, SideOp, SideFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qh, ch + 1, ch,
                           C, oph, fin, gs, never);
        hipLaunchKernelGGL((gather_fixup<GATHER_CH, SideFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qh, ch + 1, ch, fin, gs,
                           never);
        if (!walk) {
            hipLaunchKernelGGL(side_sumsq, dim3(G), dim3(GFR_BLOCK), 0, s, qh, ch + 1, x, part);
            hipLaunchKernelGGL(side_inv_norm, dim3(1), dim3(GFR_BLOCK), 0, s, part, (uint32_t)G, inv + 0);
        }
        GFR_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(side_output, dim3(G), dim3(GFR_BLOCK), 0, s, x, 0, nl, R, walk, inv + 0, iters, h0, hub_dev);
    hipLaunchKernelGGL(side_output, dim3(G), dim3(GFR_BLOCK), 0, s, x, nl, n, R, walk, inv + 1, iters, 0.0,
                       auth_dev);
    GFR_LAUNCH_CHECK();
    qb.check(c, s, walk ? "salsa" : "hits");
    deliver(c, hub, hub_dev, 8ull * nl, s);
    deliver(c, auth, auth_dev, 8ull * (n - nl), s);
    c.stats.v["iterations"] = iters;
}

}  // namespace gfr
