// bfs.hip -- single-source BFS: level-synchronous advance + filter with a
// per-level push/pull choice (Sec. 4.5 "Push vs. pull traversal", Sec. 5.1).
//
// One kernel launch per level.  The level's direction, frontier size and edge
// count live in a device control block that the last work-group of each level
// rewrites, so the host can enqueue levels speculatively and only reads a
// single word back every few launches.
//
// Push level (advance + filter fused): the frontier queue carries the exclusive
// scan of its degrees and a chunk index, so every work-group takes an equal
// slice of the frontier's edges (load-balanced partitioning, Sec. 4.4); each
// edge tests the visited bitmap and claims the neighbour with one atomicOr
// (the non-idempotent advance of Sec. 4.5), the winner writes depth and
// appends the vertex to the next queue with one 64-bit atomic per wave.
//
// Pull level: every unvisited vertex scans its neighbour list until it finds
// one in the current frontier bitmap (Sec. 4.5).  A wave owns 64 consecutive
// vertices, i.e. two whole bitmap words, so visited / next-frontier words are
// written with plain stores.
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { DIR_PUSH = 0, DIR_PULL = 1, DIR_DONE = 2 };

struct BfsCtl {
    unsigned long long next;       // packed counter of the queue being built (entries<<32 | edges)
    unsigned long long mu;         // edges incident to unvisited vertices
    unsigned long long inspected;  // edges inspected so far
    uint32_t dir;                  // DIR_* of the current level (first word read back by the host)
    uint32_t nf;                   // entries of the current queue
    uint32_t mf;                   // edges of the current queue
    int32_t level;                 // depth of the current frontier
    uint32_t cur;                  // parity of the current queue
    uint32_t arrive;               // last-work-group counter
    uint32_t nu;                   // unvisited vertices
    uint32_t force;                // 0 auto, 1 push only, 2 pull only
    float alpha, beta;
    uint32_t push_levels, pull_levels;
};

struct BfsArgs {
    const int32_t *R;
    const int32_t *C;
    int32_t n;
    uint32_t nwords;
    int32_t *depth;
    uint32_t *vis;
    uint32_t *fb[3];
    FrontierQ q[2];
    BfsCtl *ctl;
};

__device__ __forceinline__ uint32_t *pick3(const BfsArgs &a, int i)
{
    return i == 0 ? a.fb[0] : (i == 1 ? a.fb[1] : a.fb[2]);
}

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void bfs_level(BfsArgs a)
{
    BfsCtl *ctl = a.ctl;
    const uint32_t dir = ctl->dir;
    if (dir == DIR_DONE) return;
    const int32_t L = ctl->level;
    const uint32_t cur = ctl->cur;
    const FrontierQ qin = a.q[cur], qout = a.q[cur ^ 1];
    uint32_t *fb_cur = pick3(a, L % 3), *fb_next = pick3(a, (L + 1) % 3), *fb_clr = pick3(a, (L + 2) % 3);

    // the bitmap of level L+2 must be empty before level L+1 starts writing it
    for (uint32_t i = blockIdx.x * GFR_BLOCK + threadIdx.x; i < a.nwords; i += gridDim.x * GFR_BLOCK)
        fb_clr[i] = 0u;

    if (dir == DIR_PUSH) {
        __shared__ uint32_t s_off[CH + 1];
        __shared__ int32_t s_row[CH + 1];
        const uint32_t mf = ctl->mf, nf = ctl->nf;
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
#pragma unroll 1
            for (uint32_t k = 0; k < (uint32_t)CH; k += GFR_BLOCK) {
                const uint32_t e = e0 + k + threadIdx.x;
                const bool valid = e < e1;
                int32_t v = 0, rv = 0;
                uint32_t dv = 0;
                bool won = false;
                if (valid) {
                    const int i = upper_index(s_off, 0, cnt - 1, e);
                    v = a.C[s_row[i] + (int32_t)(e - s_off[i])];
                    const uint32_t bit = 1u << (v & 31);
                    uint32_t *w = a.vis + (v >> 5);
                    if (!(*w & bit)) won = !(atomicOr(w, bit) & bit);
                    if (won) {
                        a.depth[v] = L + 1;
                        atomicOr(fb_next + (v >> 5), bit);
                        rv = a.R[v];
                        dv = (uint32_t)(a.R[v + 1] - rv);
                    }
                }
                wave_enqueue(won, v, dv, rv, &ctl->next, qout, CH);
            }
        }
    } else {
        const uint32_t waves = gridDim.x * GFR_WAVES;
        const int lane = lane_id();
        uint32_t insp = 0;
        for (uint32_t grp = blockIdx.x * GFR_WAVES + threadIdx.x / 64; grp * 64u < (uint32_t)a.n;
             grp += waves) {
            const int32_t v = (int32_t)(grp * 64u) + lane;
            const uint32_t word = grp * 2u + (uint32_t)(lane >> 5);
            const bool inr = v < a.n;
            const uint32_t visw = a.vis[word];
            const bool todo = inr && !(visw & (1u << (v & 31)));
            bool found = false;
            int32_t rv = 0, re = 0;
            if (todo) {
                rv = a.R[v];
                re = a.R[v + 1];
                for (int32_t e = rv; e < re; ++e) {
                    const int32_t u = a.C[e];
                    ++insp;
                    if (fb_cur[u >> 5] & (1u << (u & 31))) {
                        found = true;
                        break;
                    }
                }
            }
            const uint64_t fm = ballot(found);
            if (found) a.depth[v] = L + 1;
            if ((lane & 31) == 0) {
                const uint32_t bits = (uint32_t)(fm >> lane);
                fb_next[word] = bits;
                if (bits) a.vis[word] = visw | bits;
            }
            wave_enqueue(found, v, (uint32_t)(re - rv), rv, &ctl->next, qout, CH);
        }
        const uint32_t tot = wave_sum_u32(insp);
        if (lane == 0 && tot) atomicAdd(&ctl->inspected, (unsigned long long)tot);
    }

    if (last_block_arrives(&ctl->arrive) && threadIdx.x == 0) {
        const unsigned long long nx = atomicAdd(&ctl->next, 0ull);
        const uint32_t nf2 = (uint32_t)(nx >> 32), mf2 = (uint32_t)nx;
        if (dir == DIR_PUSH) {
            ctl->push_levels += 1;
            ctl->inspected += ctl->mf;
        } else {
            ctl->pull_levels += 1;
        }
        ctl->nu -= nf2;
        ctl->mu -= mf2;
        uint32_t nd;
        if (nf2 == 0) nd = DIR_DONE;
        else if (ctl->force == 1) nd = DIR_PUSH;
        else if (ctl->force == 2) nd = DIR_PULL;
        else if (dir == DIR_PUSH)
            nd = ((double)mf2 > (double)ctl->mu / ctl->alpha && nf2 > ctl->nf) ? DIR_PULL : DIR_PUSH;
        else
            nd = ((double)nf2 < (double)a.n / ctl->beta && nf2 < ctl->nf) ? DIR_PUSH : DIR_PULL;
        ctl->nf = nf2;
        ctl->mf = mf2;
        ctl->next = 0ull;
        ctl->level = L + 1;
        ctl->cur = cur ^ 1u;
        ctl->dir = nd;
    }
}

__global__ void bfs_init(BfsArgs a, int32_t src, uint32_t chunk, uint32_t force, float alpha,
                         float beta, unsigned long long m)
{
    const int32_t rs = a.R[src], deg = a.R[src + 1] - rs;
    if (threadIdx.x == 0) {
        BfsCtl *ctl = a.ctl;
        a.depth[src] = 0;
        a.vis[src >> 5] = 1u << (src & 31);
        a.fb[0][src >> 5] = 1u << (src & 31);
        a.q[0].v[0] = src;
        a.q[0].off[0] = 0;
        a.q[0].row[0] = rs;
        ctl->next = 0ull;
        ctl->mu = m - (unsigned long long)deg;
        ctl->inspected = 0ull;
        ctl->nf = 1;
        ctl->mf = (uint32_t)deg;
        ctl->level = 0;
        ctl->cur = 0;
        ctl->arrive = 0;
        ctl->nu = (uint32_t)a.n - 1u;
        ctl->force = force;
        ctl->alpha = alpha;
        ctl->beta = beta;
        ctl->push_levels = ctl->pull_levels = 0;
        ctl->dir = deg == 0 ? DIR_DONE : (force == 2 ? DIR_PULL : DIR_PUSH);
    }
    for (uint32_t c = threadIdx.x; (uint64_t)c * chunk < (uint64_t)deg; c += blockDim.x) a.q[0].part[c] = 0;
}

void run_bfs(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s)
{
    const int32_t n = g.n;
    const uint32_t chunk = (uint32_t)c.opt.advance_chunk;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    size_t need = 4 * al256(nwords * 4ull) + 2 * (3 * al256(4ull * n) + al256(4 * nparts)) + al256(sizeof(BfsCtl));
    c.arena.reserve(need);
    BfsArgs a;
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.n = n;
    a.nwords = nwords;
    a.depth = depth;
    a.vis = c.arena.take<uint32_t>(nwords);
    for (int i = 0; i < 3; ++i) a.fb[i] = c.arena.take<uint32_t>(nwords);
    for (int i = 0; i < 2; ++i) {
        a.q[i].v = c.arena.take<int32_t>(n);
        a.q[i].off = c.arena.take<uint32_t>(n);
        a.q[i].row = c.arena.take<int32_t>(n);
        a.q[i].part = c.arena.take<int32_t>(nparts);
    }
    a.ctl = c.arena.take<BfsCtl>(1);

    fill_u32(depth, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.vis, 0u, nwords, s);
    fill_u32(a.fb[0], 0u, nwords, s);
    fill_u32(a.fb[1], 0u, nwords, s);
    hipLaunchKernelGGL(bfs_init, dim3(1), dim3(GFR_BLOCK), 0, s, a, src, chunk,
                       (uint32_t)c.opt.bfs_direction, (float)c.opt.bfs_alpha, (float)c.opt.bfs_beta,
                       (unsigned long long)g.m);
    GFR_LAUNCH_CHECK();

    const int G = grid_blocks(c, 4);
    auto launch = [&]() { c.ktimer.run("bfs_level", s, [&]() {
        switch (chunk) {
        case 256: hipLaunchKernelGGL(bfs_level<256>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 512: hipLaunchKernelGGL(bfs_level<512>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 1024: hipLaunchKernelGGL(bfs_level<1024>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 2048: hipLaunchKernelGGL(bfs_level<2048>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        default: hipLaunchKernelGGL(bfs_level<4096>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        }
    }); };
    const int32_t launched = run_until_done(c, &a.ctl->dir, DIR_DONE, g.bfs_levels_hint + 1,
                                            (int64_t)n + 4, s, launch);
    BfsCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(BfsCtl));
    c.stats.v["levels"] = h.level;
    c.stats.v["push_levels"] = h.push_levels;
    c.stats.v["pull_levels"] = h.pull_levels;
    c.stats.v["edges_inspected"] = (double)h.inspected;
    c.stats.v["launches"] = launched;
    g.bfs_levels_hint = h.level;
}

}  // namespace gfr
