// bc.hip -- betweenness centrality from a set of sources, Brandes'
// two-pass formulation as the paper maps it (Sec. 5.3):
//   forward   an advance identical to BFS discovers level L+1 from level L,
//             pushing from the level's lists or, when the level is large,
//             pulling: every unvisited vertex scans its own list for a vertex
//             of level L (the direction choice of Sec. 4.5, which the paper
//             names as the missing piece of its BC); then a compute step
//             gathers sigma(v) = sum of sigma(u) over the neighbours u one
//             level up (shortest-path counts, FP64);
//   backward  walks the levels in reverse and gathers
//             delta(v) = sigma(v) * sum over neighbours w one level down of
//                        (1 + delta(w)) / sigma(w),
//             stored in FP32; bc(v) accumulates delta(v) over sources.
// Both gathers are pull-style: no floating-point atomics, fixed order per
// list (see gather.h).  Depths are kept as one byte per vertex, depth mod
// 128 (0xFF = unvisited): the neighbours a gather inspects are within one
// level of the gathering vertex (or not yet discovered), so the byte
// identifies the level exactly, and the array is a quarter of an int32 one,
// which keeps the random probes of the gathers in cache.  Every level is kept as a contiguous slice of one BFS
// order array so the backward pass can revisit it.
#include <vector>

#include "compact.h"
#include "engine.h"
#include "gather.h"

namespace gfr {

constexpr uint8_t BC_UNSEEN = 0xFF;   // never a level code

__host__ __device__ __forceinline__ uint8_t level_code(int32_t L) { return (uint8_t)(L & 127); }
static_assert(BC_UNSEEN > 127, "unvisited must differ from every level code");

struct BcArgs {
    const int32_t *R;
    const int32_t *C;
    uint8_t *dc;     // depth code per vertex
    uint32_t *vis;
};

// push advance of one level (load-balanced edge chunks): an unvisited
// neighbour gets its depth code and a mark byte (plain stores; duplicates write
// the same values and collapse in the compaction)
template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void bc_discover(BcArgs a, FrontierQ qin, uint32_t nf, uint32_t mf,
                                                         int32_t L, uint8_t *mark)
{
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    const uint32_t nchunks = (mf + CH - 1) / CH;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t e0 = c * CH;
        const uint32_t e1 = min(e0 + (uint32_t)CH, mf);
        const int s = qin.part[c];
        const int t = (c + 1 < nchunks) ? qin.part[c + 1] : (int)nf - 1;
        const int cnt = t - s + 1;
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            s_off[i] = qin.off[s + i];
            s_row[i] = qin.row[s + i];
        }
        __syncthreads();
        for (uint32_t k = 0; k < (uint32_t)CH; k += GFR_BLOCK) {
            const uint32_t e = e0 + k + threadIdx.x;
            if (e < e1) {
                const int i = upper_index(s_off, 0, cnt - 1, e);
                const int32_t v = a.C[s_row[i] + (int32_t)(e - s_off[i])];
                if (!((a.vis[v >> 5] >> (v & 31)) & 1u) && !mark[v]) {
                    a.dc[v] = level_code(L + 1);
                    mark[v] = 1;
                }
            }
        }
    }
}

// pull discovery of level L+1: every unvisited vertex (lane = vertex) scans
// its list four neighbours at a time until one is in the level-L bitmap
__global__ __launch_bounds__(GFR_BLOCK) void bc_pull_discover(BcArgs a, int32_t n, const uint32_t *fb, int32_t L,
                                                              uint8_t *mark)
{
    const uint32_t waves = gridDim.x * GFR_WAVES;
    const int lane = lane_id();
    for (uint32_t grp = blockIdx.x * GFR_WAVES + threadIdx.x / 64; grp * 64u < (uint32_t)n; grp += waves) {
        const int32_t v = (int32_t)(grp * 64u) + lane;
        const uint32_t visw = a.vis[grp * 2u + (uint32_t)(lane >> 5)];
        bool found = false;
        if (v < n && !(visw & (1u << (v & 31)))) {
            int32_t e = a.R[v];
            const int32_t re = a.R[v + 1];
            while (e < re) {
                const int32_t k = min(4, re - e);
                int32_t u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) u[j] = a.C[j < k ? e + j : e];
                uint32_t hit = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) hit |= (j < k) ? (fb[u[j] >> 5] >> (u[j] & 31)) & 1u : 0u;
                if (hit) {
                    found = true;
                    break;
                }
                e += 4;
            }
        }
        if (found) {
            a.dc[v] = level_code(L + 1);
            mark[v] = 1;
        }
    }
}

// compaction of one BFS level into its slice of the BFS order (vertex order);
// also writes the level's bitmap for a following pull discovery
struct BcMarks {
    uint8_t *mark;
    uint32_t *vis;
    uint32_t *fb;
    unsigned long long *out;   // packed (entries << 32 | edges) of the new level
    uint32_t *parity;
    __device__ bool skip() const { return false; }
    __device__ uint32_t mask(uint32_t w) const
    {
        const uint32_t m = marks_to_mask(mark + 32ull * w);
        if (m) {
            clear_marks(mark + 32ull * w);
            vis[w] |= m;
        }
        fb[w] = m;
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

__global__ void bc_source_init(BcArgs a, int32_t src, FrontierQ q0, double *sigma, unsigned long long *ctr0,
                               uint32_t *fb)
{
    const int32_t rs = a.R[src], deg = a.R[src + 1] - rs;
    if (threadIdx.x == 0) {
        a.dc[src] = level_code(0);
        a.vis[src >> 5] |= 1u << (src & 31);
        fb[src >> 5] |= 1u << (src & 31);
        sigma[src] = 1.0;
        q0.v[0] = src;
        q0.off[0] = 0;
        q0.row[0] = rs;
        *ctr0 = (1ull << 32) | (unsigned long long)(uint32_t)deg;
    }
    for (uint32_t c = threadIdx.x; (uint64_t)c * GATHER_CH < (uint64_t)deg; c += blockDim.x) q0.part[c] = 0;
}

struct SigmaOp {
    const uint8_t *dc;
    const double *sigma;
    uint8_t code;   // level of the predecessors
    __device__ double operator()(int32_t u, int32_t) const { return dc[u] == code ? sigma[u] : 0.0; }
};

struct SigmaFin {
    double *sigma;
    __device__ void operator()(int32_t v, double s) const { sigma[v] = s; }
};

struct DeltaOp {
    const uint8_t *dc;
    const double *coef;
    uint8_t code;   // level of the successors
    __device__ double operator()(int32_t w, int32_t) const { return dc[w] == code ? coef[w] : 0.0; }
};

struct DeltaFin {
    const double *sigma;
    double *coef;
    double *bc;
    __device__ void operator()(int32_t v, double s) const
    {
        const float dl = (float)(sigma[v] * s);
        coef[v] = (1.0 + (double)dl) / sigma[v];
        bc[v] += (double)dl;
    }
};

__global__ void bc_leaf_coef(const FrontierQ q, uint32_t nf, const double *sigma, double *coef)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) {
        const int32_t v = q.v[i];
        coef[v] = 1.0 / sigma[v];
    }
}

__global__ void bc_to_f32(const double *acc, float *out, int32_t n)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        out[v] = (float)acc[v];
}

struct Level {
    uint32_t start, nf, mf, pbase;
};

void run_bc(Ctx &c, Graph &g, const int32_t *sources, int32_t k, float *bc, hipStream_t s)
{
    const int32_t n = g.n;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / GATHER_CH) + 2ull * n + 4;
    const size_t nch = (size_t)(g.m / GATHER_CH) + 2;
    const size_t nlev = (size_t)n + 2;
    c.arena.reserve(al256(4ull * n) + al256(4ull * nwords) + al256(32ull * nwords) + 3 * al256(8ull * n) + 3 * al256(4ull * n) +
                    al256(4 * nparts) + 2 * al256(8 * nch) + al256(8 * nlev) +
                    al256(16ull * (uint64_t)compact_geom(nwords, c.num_cu).blocks) + al256(256) +
                    al256(4ull * nwords));
    BcArgs a;
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.dc = c.arena.take<uint8_t>(4ull * ((n + 3) / 4));
    a.vis = c.arena.take<uint32_t>(nwords);
    double *sigma = c.arena.take<double>(n);
    double *coef = c.arena.take<double>(n);
    double *acc = c.arena.take<double>(n);
    int32_t *order = c.arena.take<int32_t>(n);
    uint32_t *off = c.arena.take<uint32_t>(n);
    int32_t *row = c.arena.take<int32_t>(n);
    int32_t *part = c.arena.take<int32_t>(nparts);
    GatherScratch gs{c.arena.take<double>(nch), c.arena.take<double>(nch)};
    unsigned long long *ctr = c.arena.take<unsigned long long>(nlev);
    const int G = grid_blocks(c, 4);
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    uint8_t *mark = c.arena.take<uint8_t>(32ull * nwords);
    unsigned long long *status = c.arena.take<unsigned long long>(2ull * cg.blocks);
    uint32_t *cw = c.arena.take<uint32_t>(64);   // [0] compaction parity, [1] look-back error
    uint32_t *fb = c.arena.take<uint32_t>(nwords);
    fill_u32(mark, 0u, 8ull * nwords, s);
    fill_u32(status, 0u, 4ull * cg.blocks, s);
    fill_u32(cw, 0u, 64, s);

    fill_u32(acc, 0u, 2ull * n, s);
    auto qat = [&](const Level &l) {
        return FrontierQ{order + l.start, off + l.start, row + l.start, part + l.pbase};
    };
    std::vector<Level> lv;
    double levels_total = 0, push_levels = 0, pull_levels = 0;
    const int force = c.opt.bc_direction;
    const double alpha = c.opt.bc_alpha, beta = c.opt.bc_beta;
    for (int32_t si = 0; si < k; ++si) {
        const int32_t src = sources[si];
        fill_u32(a.dc, 0xFFFFFFFFu, (n + 3) / 4, s);   // BC_UNSEEN
        fill_u32(a.vis, 0u, nwords, s);
        fill_u32(fb, 0u, nwords, s);
        lv.clear();
        lv.push_back(Level{0, 1, 0, 0});
        hipLaunchKernelGGL(bc_source_init, dim3(1), dim3(GFR_BLOCK), 0, s, a, src, qat(lv[0]), sigma, ctr, fb);
        GFR_LAUNCH_CHECK();
        GFR_HIP(hipMemcpyAsync(c.pinned, ctr, 8, hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        lv[0].mf = c.pinned[0];
        // unvisited vertices and their edges, for the direction choice
        double mu = (double)g.m - (double)lv[0].mf, prev_nf = 0.0;
        bool pull = false;
        // forward
        for (;;) {
            const Level cur = lv.back();
            const int32_t L = (int32_t)lv.size() - 1;
            if (cur.mf == 0) break;
            if (force == 1) pull = false;
            else if (force == 2) pull = true;
            else if (!pull) pull = (double)cur.mf > mu / alpha && (double)cur.nf > prev_nf;
            else pull = !((double)cur.nf < (double)n / beta && (double)cur.nf < prev_nf);
            prev_nf = (double)cur.nf;
            Level nx{cur.start + cur.nf, 0, 0, cur.pbase + (cur.mf + GATHER_CH - 1) / GATHER_CH + 1};
            unsigned long long *cn = ctr + lv.size();
            if (pull) {
                hipLaunchKernelGGL(bc_pull_discover, dim3(G), dim3(GFR_BLOCK), 0, s, a, n, fb, L, mark);
                pull_levels += 1;
            } else {
                hipLaunchKernelGGL(bc_discover<GATHER_CH>, dim3(G), dim3(GFR_BLOCK), 0, s, a, qat(cur), cur.nf,
                                   cur.mf, L, mark);
                push_levels += 1;
            }
            hipLaunchKernelGGL(compact_kernel<BcMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, a.R, n, nwords, cg.wpt,
                               BcMarks{mark, a.vis, fb, cn, cw}, qat(nx), GATHER_CH, status, cw, cw + 1);
            GFR_LAUNCH_CHECK();
            GFR_HIP(hipMemcpyAsync(c.pinned, cn, 8, hipMemcpyDeviceToHost, s));
            GFR_HIP(hipStreamSynchronize(s));
            nx.mf = c.pinned[0];
            nx.nf = c.pinned[1];
            if (nx.nf == 0) break;
            mu -= (double)nx.mf;
            lv.push_back(nx);
            const uint32_t *cw = (const uint32_t *)cn;
            hipLaunchKernelGGL((gather_chunks<GATHER_CH, SigmaOp, SigmaFin>), dim3(G), dim3(GFR_BLOCK), 0, s,
                               qat(nx), cw + 1, cw, a.C, SigmaOp{a.dc, sigma, level_code(L)}, SigmaFin{sigma}, gs,
                               c.zero_word.as<uint32_t>());
            hipLaunchKernelGGL((gather_fixup<GATHER_CH, SigmaFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qat(nx), cw + 1,
                               cw, SigmaFin{sigma}, gs, c.zero_word.as<uint32_t>());
            GFR_LAUNCH_CHECK();
        }
        levels_total += (double)lv.size();
        // backward: deepest level has no successors
        const int32_t Lmax = (int32_t)lv.size() - 1;
        if (Lmax >= 1) {
            const Level &d = lv[Lmax];
            hipLaunchKernelGGL(bc_leaf_coef, dim3(G), dim3(GFR_BLOCK), 0, s, qat(d), d.nf, sigma, coef);
            GFR_LAUNCH_CHECK();
        }
        for (int32_t L = Lmax - 1; L >= 1; --L) {
            const Level &l = lv[L];
            const uint32_t *cw = (const uint32_t *)(ctr + L);
            hipLaunchKernelGGL((gather_chunks<GATHER_CH, DeltaOp, DeltaFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qat(l),
                               cw + 1, cw, a.C, DeltaOp{a.dc, coef, level_code(L + 1)}, DeltaFin{sigma, coef, acc}, gs,
                               c.zero_word.as<uint32_t>());
            hipLaunchKernelGGL((gather_fixup<GATHER_CH, DeltaFin>), dim3(G), dim3(GFR_BLOCK), 0, s, qat(l), cw + 1, cw,
                               DeltaFin{sigma, coef, acc}, gs, c.zero_word.as<uint32_t>());
            GFR_LAUNCH_CHECK();
        }
    }
    hipLaunchKernelGGL(bc_to_f32, dim3(G), dim3(GFR_BLOCK), 0, s, acc, bc, n);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, cw + 1, 4, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    if (c.pinned[0]) fail(GFR_E_DEVICE, "bc: frontier compaction look-back timed out");
    c.stats.v["levels"] = levels_total;
    c.stats.v["push_levels"] = push_levels;
    c.stats.v["pull_levels"] = pull_levels;
}

}  // namespace gfr
