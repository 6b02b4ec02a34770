// bfs.hip -- single-source BFS: level-synchronous advance + filter with a
// per-level push/pull choice (Sec. 4.5 "Push vs. pull traversal", Sec. 5.1).
//
// Every level is two launches:
//   bfs_level   the advance.  Push: the frontier queue carries the exclusive
//               scan of its degrees and a chunk index, so every work-group
//               takes an equal slice of the frontier's edges (load-balanced
//               partitioning, Sec. 4.4); each edge tests the visited bitmap
//               and, for an unvisited neighbour not yet marked, writes its
//               depth and a mark byte with plain stores.  This is the
//               idempotent advance of Sec. 4.5: concurrent discoverers write
//               the same values, and the compaction removes the duplicates.
//               (With bfs.dedup = 0 the neighbour is first claimed with an
//               atomicOr on the visited bitmap, the non-idempotent form.)
//               Pull: every unvisited vertex scans its list until it meets a
//               vertex of the current frontier bitmap.
//               Either way the new frontier is a byte array of marks.
//   compact     the filter: the marks become the next queue in vertex order
//               and the next frontier bitmap, visited is updated (compact.h),
//               and the last work-group runs the level control:
//               stop on an empty frontier, otherwise choose push or pull from
//               the frontier's edge count against the unvisited vertices'
//               (the rule of Sec. 4.5, with tunable ratios alpha and beta).
// The control state lives in device memory, so the host enqueues levels
// speculatively and only reads one word back every few levels.
//
// On mesh-like graphs (small, even degrees, long diameters) the frontier is
// kept as mark bytes only, with one launch per level (bfs_bitmap_level): each
// thread scans 16 mark bytes of the current level, consumes them, and expands
// every marked vertex's list (through a per-work-group LDS list); an unvisited
// neighbour (depth still -1) gets its depth and a mark byte for the next level,
// with plain idempotent stores
// (Sec. 4.5).  There is no queue and no compaction: on such graphs a level's
// cost is the chain of memory round trips of its launches, and this halves the
// number of launches and drops the compaction's scan and look-back.  Each
// work-group records whether it marked anything; the next launch's first
// work-group reads those flags and ends the traversal when all are zero.
#include "compact.h"
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { DIR_PUSH = 0, DIR_PULL = 1, DIR_DONE = 2 };

struct BfsCtl {
    uint32_t dir;       // DIR_* of the current level (first word: read back by the host)
    int32_t level;      // depth of the current frontier
    uint32_t nf, mf;    // entries / edges of the current queue
    unsigned long long mu;  // edges incident to unvisited vertices
    uint32_t nu;        // unvisited vertices
    uint32_t force;     // 0 auto, 1 push only, 2 pull only
    uint32_t dedup;     // 0 atomic claim, 1 idempotent
    float alpha, beta;
    uint32_t parity;    // status-buffer parity of the compaction
    uint32_t err;       // compaction look-back gave up (never expected)
    uint32_t push_levels, pull_levels;
    // traffic model counters (summed over levels)
    unsigned long long push_entries, push_edges, push_new;
    unsigned long long pull_unvisited, pull_inspected, pull_new;
};

struct BfsArgs {
    const int32_t *R;
    const int32_t *C;
    int32_t n;
    uint32_t nwords;
    int32_t *depth;
    uint32_t *vis;        // visited bitmap (updated by the compaction)
    uint32_t *fb;         // current frontier bitmap (written by the compaction)
    uint8_t *mark;        // next-frontier marks, one byte per vertex
    FrontierQ q;
    uint32_t *part_insp;   // per work-group edges inspected by a pull level
    BfsCtl *ctl;
    uint32_t mapping;        // push work mapping: 0 by frontier size, 1 edge chunks, 2 per-vertex groups
    uint32_t twc_threshold;  // mapping 0: per-vertex groups below this many frontier vertices
};

// One push edge of BFS level L: test the visited bit, claim (or, idempotent,
// just write) an unvisited target's depth and next-frontier mark.
__device__ __forceinline__ void bfs_push_edge(const BfsArgs &a, int32_t v, int32_t L, bool idem)
{
    const uint32_t bit = 1u << (v & 31);
    uint32_t *w = a.vis + (v >> 5);
    if (!(*w & bit) && !a.mark[v]) {
        if (idem || !(atomicOr(w, bit) & bit)) {
            a.depth[v] = L + 1;
            a.mark[v] = 1;
        }
    }
}

// The per-vertex mapping of Sec. 4.4 (per-CTA / per-warp coarse-grained,
// then the fine-grained strategy for the rest): each work-group takes
// GFR_BLOCK frontier vertices, one per thread.  Lists of at least GFR_BLOCK
// edges are taken one at a time by the whole work-group (their owners compete
// for it through an LDS word), then lists of at least 64 edges one at a time
// by the owner's wave.  The remaining short lists are processed by the whole
// work-group together: their sizes are scanned, the list offsets sit in LDS,
// and each thread takes every GFR_BLOCK-th of their edges, finding its list
// by binary search (the cooperative fine-grained form of Sec. 4.4).
__device__ void bfs_push_twc(const BfsArgs &a, const FrontierQ &q, uint32_t nf, uint32_t mf, int32_t L, bool idem)
{
    __shared__ int32_t s_owner, s_row, s_deg;
    __shared__ uint32_t s_soff[GFR_BLOCK + 1];
    __shared__ int32_t s_srow[GFR_BLOCK];
    __shared__ uint32_t s_wsum[GFR_WAVES];
    const int lane = lane_id(), wave = threadIdx.x / 64;
    for (uint32_t base = blockIdx.x * GFR_BLOCK; base < nf; base += gridDim.x * GFR_BLOCK) {
        const uint32_t i = base + threadIdx.x;
        int32_t row = 0, deg = 0;
        if (i < nf) {
            row = q.row[i];
            deg = (int32_t)((i + 1 < nf ? q.off[i + 1] : mf) - q.off[i]);
        }
        for (;;) {   // work-group lists
            if (threadIdx.x == 0) s_owner = -1;
            __syncthreads();
            if (deg >= GFR_BLOCK) s_owner = (int32_t)threadIdx.x;   // one of the writers wins
            __syncthreads();
            const int32_t owner = s_owner;
            if (owner < 0) break;
            if ((int32_t)threadIdx.x == owner) {
                s_row = row;
                s_deg = deg;
                deg = 0;
            }
            __syncthreads();
            const int32_t r0 = s_row, d0 = s_deg;
            for (int32_t k = (int32_t)threadIdx.x; k < d0; k += GFR_BLOCK) bfs_push_edge(a, a.C[r0 + k], L, idem);
            __syncthreads();   // s_row / s_deg are rewritten by the next owner
        }
        for (;;) {   // wave lists
            const uint64_t want = ballot(deg >= 64);
            if (!want) break;
            const int src = __ffsll((unsigned long long)want) - 1;
            const int32_t r0 = __builtin_amdgcn_readlane(row, src), d0 = __builtin_amdgcn_readlane(deg, src);
            if (lane == src) deg = 0;
            for (int32_t k = lane; k < d0; k += 64) bfs_push_edge(a, a.C[r0 + k], L, idem);
        }
        // short lists, the whole work-group over their concatenated edges
        const uint32_t incl = wave_incl_scan((uint32_t)deg);
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        uint32_t wbase = 0, total = 0;
        for (int k = 0; k < GFR_WAVES; ++k) {
            if (k < wave) wbase += s_wsum[k];
            total += s_wsum[k];
        }
        s_soff[threadIdx.x] = wbase + incl - (uint32_t)deg;
        s_srow[threadIdx.x] = row;
        if (threadIdx.x == 0) s_soff[GFR_BLOCK] = total;
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < total; e += GFR_BLOCK) {
            const int j = upper_index(s_soff, 0, GFR_BLOCK - 1, e);   // lists of size 0 share offsets: the last wins
            bfs_push_edge(a, a.C[s_srow[j] + (int32_t)(e - s_soff[j])], L, idem);
        }
        __syncthreads();   // LDS is reused by the next slice
    }
}

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void bfs_level(BfsArgs a)
{
    BfsCtl *ctl = a.ctl;
    const uint32_t dir = ctl->dir;
    if (dir == DIR_DONE) return;
    const int32_t L = ctl->level;

    if (dir == DIR_PUSH) {
        __shared__ uint32_t s_off[CH + 1];
        __shared__ int32_t s_row[CH + 1];
        const uint32_t mf = ctl->mf, nf = ctl->nf;
        const bool idem = ctl->dedup != 0;
        const FrontierQ q = a.q;
        // Sec. 4.4's hybrid: per-vertex groups for frontiers below the
        // threshold, equal edge chunks (load-balanced partitioning) above it
        if (a.mapping == 2 || (a.mapping == 0 && nf < a.twc_threshold)) {
            bfs_push_twc(a, q, nf, mf, L, idem);
            return;
        }
        const uint32_t nchunks = (mf + CH - 1) / CH;
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
            }
            __syncthreads();
            // each thread takes every GFR_BLOCK-th edge of the chunk: all its
            // column loads are issued first, then all visited-word probes,
            // then the tests (an edge past the chunk end repeats the chunk's
            // first edge and is masked)
            constexpr int PER = CH / GFR_BLOCK;
            int32_t vv[PER];
            uint32_t vw[PER];
            bool ok[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const uint32_t e = e0 + p * GFR_BLOCK + threadIdx.x;
                ok[p] = e < e1;
                const uint32_t ec = ok[p] ? e : e0;
                const int i = upper_index(s_off, 0, cnt - 1, ec);
                vv[p] = a.C[s_row[i] + (int32_t)(ec - s_off[i])];
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) vw[p] = a.vis[vv[p] >> 5];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int32_t v = vv[p];
                const uint32_t bit = 1u << (v & 31);
                if (ok[p] && !(vw[p] & bit) && !a.mark[v]) {
                    if (idem || !(atomicOr(a.vis + (v >> 5), bit) & bit)) {
                        a.depth[v] = L + 1;
                        a.mark[v] = 1;
                    }
                }
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
            const uint32_t visw = a.vis[word];
            bool found = false;
            if (v < a.n && !(visw & (1u << (v & 31)))) {
                int32_t e = a.R[v];
                const int32_t re = a.R[v + 1];
                // four independent neighbour probes per step
                while (e < re) {
                    const int32_t k = min(4, re - e);
                    int32_t u[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) u[j] = a.C[j < k ? e + j : e];
                    uint32_t hit = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) hit |= (j < k) ? (a.fb[u[j] >> 5] >> (u[j] & 31)) & 1u : 0u;
                    insp += (uint32_t)k;
                    if (hit) {
                        found = true;
                        break;
                    }
                    e += 4;
                }
            }
            if (found) {
                a.depth[v] = L + 1;
                a.mark[v] = 1;
            }
        }
        // per-group partial (plain store, summed by the level control)
        __shared__ uint32_t s_insp[GFR_WAVES];
        const uint32_t tot = wave_sum_u32(insp);
        if (lane == 0) s_insp[threadIdx.x / 64] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int i = 0; i < GFR_WAVES; ++i) t += s_insp[i];
            a.part_insp[blockIdx.x] = t;
        }
    }
}

// Filter + level control for the compaction kernel.
struct BfsMarks {
    BfsArgs a;
    uint32_t nparts;   // work-groups of bfs_level (entries of part_insp)

    __device__ bool skip() const { return a.ctl->dir == DIR_DONE; }
    __device__ uint32_t mask(uint32_t w) const
    {
        const uint32_t m = marks_to_mask(a.mark + 32ull * w);
        if (m) {
            clear_marks(a.mark + 32ull * w);
            a.vis[w] |= m;
        }
        a.fb[w] = m;
        return m;
    }
    __device__ void partial(uint32_t) {}
    __device__ void control(uint32_t nf2, uint32_t mf2) const
    {
        BfsCtl *ctl = a.ctl;
        const uint32_t dir = ctl->dir;
        uint32_t insp = 0;
        if (dir == DIR_PULL) {
            for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) insp += a.part_insp[i];
            __shared__ uint32_t s[GFR_WAVES];
            insp = wave_sum_u32(insp);
            if (lane_id() == 0) s[threadIdx.x / 64] = insp;
            __syncthreads();
            insp = 0;
            for (int i = 0; i < GFR_WAVES; ++i) insp += s[i];
        }
        if (threadIdx.x != 0) return;
        if (dir == DIR_PUSH) {
            ctl->push_levels += 1;
            ctl->push_entries += ctl->nf;
            ctl->push_edges += ctl->mf;
            ctl->push_new += nf2;
        } else {
            ctl->pull_levels += 1;
            ctl->pull_unvisited += ctl->nu;
            ctl->pull_inspected += insp;
            ctl->pull_new += nf2;
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
        ctl->level += 1;
        ctl->parity ^= 1u;
        ctl->dir = nd;
    }
};

__global__ void bfs_init(BfsArgs a, int32_t src, uint32_t chunk, uint32_t force, uint32_t dedup, float alpha,
                         float beta, unsigned long long m)
{
    const int32_t rs = a.R[src], deg = a.R[src + 1] - rs;
    if (threadIdx.x == 0) {
        BfsCtl *ctl = a.ctl;
        a.depth[src] = 0;
        a.vis[src >> 5] = 1u << (src & 31);
        a.fb[src >> 5] = 1u << (src & 31);
        a.q.v[0] = src;
        a.q.off[0] = 0;
        a.q.row[0] = rs;
        ctl->mu = m - (unsigned long long)deg;
        ctl->nf = 1;
        ctl->mf = (uint32_t)deg;
        ctl->level = 0;
        ctl->nu = (uint32_t)a.n - 1u;
        ctl->force = force;
        ctl->dedup = dedup;
        ctl->alpha = alpha;
        ctl->beta = beta;
        ctl->parity = 0;
        ctl->err = 0;
        ctl->push_levels = ctl->pull_levels = 0;
        ctl->push_entries = ctl->push_edges = ctl->push_new = 0ull;
        ctl->pull_unvisited = ctl->pull_inspected = ctl->pull_new = 0ull;
        ctl->dir = deg == 0 ? DIR_DONE : (force == 2 ? DIR_PULL : DIR_PUSH);
    }
    for (uint32_t c = threadIdx.x; (uint64_t)c * chunk < (uint64_t)deg; c += blockDim.x) a.q.part[c] = 0;
}

struct BmArgs {
    const int32_t *R;
    const int32_t *C;
    int32_t n;
    int32_t *depth;
    uint8_t *mk[2];      // mark bytes of the frontier, by level parity (n rounded up to 16 bytes)
    uint32_t *flags;     // [2][gridDim]: did the work-group mark a vertex, by level parity
    BfsCtl *ctl;
};

__global__ void bfs_bitmap_init(BmArgs a, int32_t src)
{
    BfsCtl *ctl = a.ctl;
    a.depth[src] = 0;
    a.mk[0][src] = 1;
    ctl->dir = DIR_PUSH;
    ctl->level = 0;
    ctl->err = 0;
    ctl->push_levels = ctl->pull_levels = 0;
    ctl->push_entries = ctl->push_edges = ctl->push_new = 0ull;
    ctl->pull_unvisited = ctl->pull_inspected = ctl->pull_new = 0ull;
}

// level L of a mark-byte traversal (one launch per level; L is the launch index)
__global__ __launch_bounds__(GFR_BLOCK) void bfs_bitmap_level(BmArgs a, int32_t L)
{
    BfsCtl *ctl = a.ctl;
    if (ctl->dir == DIR_DONE) return;
    const uint32_t G = gridDim.x;
    uint8_t *cur = a.mk[L & 1];
    uint8_t *nxt = a.mk[(L & 1) ^ 1];
    if (L > 0 && blockIdx.x == 0) {
        // the previous level marked nothing: this level's frontier is empty
        const uint32_t *fprev = a.flags + (size_t)((L & 1) ^ 1) * G;
        uint32_t any = 0;
        for (uint32_t i = threadIdx.x; i < G; i += GFR_BLOCK) any |= fprev[i];
        if (!__syncthreads_or((int)any)) {
            if (threadIdx.x == 0) {
                ctl->level = L;
                ctl->push_levels = (uint32_t)L;
                ctl->dir = DIR_DONE;
            }
            return;
        }
    }
    // Rounds of 256 chunks of 16 mark bytes per work-group: the marked
    // vertices of a round are appended to an LDS list, then the whole group
    // expands the list, one vertex per thread, with the column and depth loads
    // of eight edges issued before any test.
    constexpr int BM_LIST = GFR_BLOCK * 16;
    __shared__ int32_t s_v[BM_LIST];
    __shared__ uint32_t s_cnt;
    int found = 0;
    const size_t nchunks = ((size_t)a.n + 15) / 16;
    for (size_t c0 = (size_t)blockIdx.x * GFR_BLOCK; c0 < nchunks; c0 += (size_t)G * GFR_BLOCK) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const size_t ci = c0 + threadIdx.x;
        if (ci < nchunks) {
            uint4 *p = (uint4 *)(cur + ci * 16);
            const uint4 w = *p;
            if ((w.x | w.y | w.z | w.w) != 0u) {
                *p = make_uint4(0u, 0u, 0u, 0u);   // consumed: clean when it next receives marks
                const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if ((ws[j >> 2] >> (8 * (j & 3))) & 0xFFu) s_v[atomicAdd(&s_cnt, 1u)] = (int32_t)(ci * 16 + j);
            }
        }
        __syncthreads();
        const uint32_t cnt = s_cnt;   // at most 16 per thread: fits BM_LIST
        for (uint32_t i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            const int32_t v = s_v[i];   // only vertices < n are ever marked
            const int32_t e1 = a.R[v + 1];
            for (int32_t e = a.R[v]; e < e1; e += 8) {
                int32_t u[8], d[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) u[k] = a.C[min(e + k, e1 - 1)];
#pragma unroll
                for (int k = 0; k < 8; ++k) d[k] = a.depth[u[k]];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (e + k < e1 && d[k] < 0) {
                        a.depth[u[k]] = L + 1;
                        nxt[u[k]] = 1;
                        found = 1;
                    }
                }
            }
        }
        __syncthreads();   // the list is reused by the next round
    }
    found = __syncthreads_or(found);
    if (threadIdx.x == 0) a.flags[(size_t)(L & 1) * G + blockIdx.x] = (uint32_t)found;
}

static void run_bfs_bitmap(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s, Arena &ar)
{
    const int32_t n = g.n;
    const size_t nb = ((size_t)n + 15) / 16 * 16;
    const int G = grid_blocks(c, 8);
    ar.reserve(2 * al256(nb) + al256(8ull * G) + al256(sizeof(BfsCtl)));
    BmArgs a;
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.n = n;
    a.depth = depth;
    a.mk[0] = ar.take<uint8_t>(nb);
    a.mk[1] = ar.take<uint8_t>(nb);
    a.flags = ar.take<uint32_t>(2ull * G);
    a.ctl = ar.take<BfsCtl>(1);
    fill_u32(depth, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.mk[0], 0u, nb / 4, s);
    fill_u32(a.mk[1], 0u, nb / 4, s);
    fill_u32(a.flags, 0u, 2ull * G, s);
    hipLaunchKernelGGL(bfs_bitmap_init, dim3(1), dim3(1), 0, s, a, src);
    GFR_LAUNCH_CHECK();
    int32_t level = 0;
    auto launch = [&]() {
        c.ktimer.run("bfs_bitmap_level", s, [&]() {
            hipLaunchKernelGGL(bfs_bitmap_level, dim3(G), dim3(GFR_BLOCK), 0, s, a, level);
        });
        ++level;
    };
    const int32_t launched = run_until_done(c, &a.ctl->dir, DIR_DONE, g.levels_hint() + 2, (int64_t)n + 4, s,
                                            launch);
    BfsCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(BfsCtl));
    c.stats.v["levels"] += h.level;
    c.stats.v["push_levels"] += h.push_levels;
    c.stats.v["pull_levels"] += 0.0;
    c.stats.v["launches"] += launched;
    c.stats.v["solves"] += 1.0;
    g.bfs_levels_hint.store(h.level, std::memory_order_relaxed);
}

void run_bfs(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s) { run_bfs(c, g, src, depth, s, c.arena); }

void run_bfs(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s, Arena &ar)
{
    // mark-byte levels on mesh-like graphs (bfs.frontier 0 auto, 1 queue, 2 mark bytes); a forced pull
    // direction needs the queue path's frontier bitmap
    const int fr = c.opt.bfs_frontier;
    if (c.opt.bfs_direction != 2 && (fr == 2 || (fr == 0 && g.cls == GRAPH_MESH))) {
        run_bfs_bitmap(c, g, src, depth, s, ar);
        return;
    }
    const int32_t n = g.n;
    const uint32_t chunk = (uint32_t)c.opt.advance_chunk;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    const int G = grid_blocks(c, 8);   // eight work-groups per CU fit at the default chunk
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    size_t need = 2 * al256(nwords * 4ull) + al256(nwords * 32ull) + 3 * al256(4ull * n) + al256(4 * nparts) +
                  al256(4ull * G) + al256(16ull * cg.blocks) + al256(sizeof(BfsCtl));
    ar.reserve(need);
    BfsArgs a;
    memset(&a, 0, sizeof a);   // padding too: the bytes key the captured steps
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.n = n;
    a.nwords = nwords;
    a.depth = depth;
    a.vis = ar.take<uint32_t>(nwords);
    a.fb = ar.take<uint32_t>(nwords);
    a.mark = ar.take<uint8_t>(32ull * nwords);
    a.q.v = ar.take<int32_t>(n);
    a.q.off = ar.take<uint32_t>(n);
    a.q.row = ar.take<int32_t>(n);
    a.q.part = ar.take<int32_t>(nparts);
    a.part_insp = ar.take<uint32_t>(G);
    a.mapping = (uint32_t)c.opt.advance_mapping;
    a.twc_threshold = (uint32_t)c.opt.twc_threshold;
    unsigned long long *status = ar.take<unsigned long long>(2ull * cg.blocks);
    a.ctl = ar.take<BfsCtl>(1);

    fill_u32(depth, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.vis, 0u, nwords, s);
    fill_u32(a.fb, 0u, nwords, s);
    fill_u32(a.mark, 0u, 8ull * nwords, s);
    fill_u32(status, 0u, 4ull * cg.blocks, s);
    hipLaunchKernelGGL(bfs_init, dim3(1), dim3(GFR_BLOCK), 0, s, a, src, chunk, (uint32_t)c.opt.bfs_direction,
                       (uint32_t)c.opt.bfs_dedup, (float)c.opt.bfs_alpha, (float)c.opt.bfs_beta,
                       (unsigned long long)g.m);
    GFR_LAUNCH_CHECK();

    BfsMarks marks{a, (uint32_t)G};
    auto launch = [&]() {
        c.ktimer.run("bfs_level", s, [&]() {
            switch (chunk) {
            case 256: hipLaunchKernelGGL(bfs_level<256>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 512: hipLaunchKernelGGL(bfs_level<512>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 1024: hipLaunchKernelGGL(bfs_level<1024>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 2048: hipLaunchKernelGGL(bfs_level<2048>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            default: hipLaunchKernelGGL(bfs_level<4096>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            }
        });
        c.ktimer.run("bfs_compact", s, [&]() {
            hipLaunchKernelGGL(compact_kernel<BfsMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, a.R, n, nwords,
                               cg.wpt, marks, a.q, chunk, status, &a.ctl->parity, &a.ctl->err);
        });
    };
    // (no captured steps over fixed scratch: instantiating a graph may allocate)
    StepKey key("bfs");
    key.add(a).add(G).add(cg).add(chunk).add(status);
    const int32_t launched = run_until_done(c, &a.ctl->dir, DIR_DONE, g.levels_hint() + 1,
                                            (int64_t)n + 4, s, launch, ar.fixed ? nullptr : &key);
    BfsCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(BfsCtl));
    if (h.err) fail(GFR_E_DEVICE, "bfs: frontier compaction look-back timed out");
    c.stats.v["levels"] += h.level;
    c.stats.v["push_levels"] += h.push_levels;
    c.stats.v["pull_levels"] += h.pull_levels;
    c.stats.v["edges_inspected"] += (double)(h.push_edges + h.pull_inspected);
    c.stats.v["push_entries"] += (double)h.push_entries;
    c.stats.v["push_edges"] += (double)h.push_edges;
    c.stats.v["push_new"] += (double)h.push_new;
    c.stats.v["pull_unvisited"] += (double)h.pull_unvisited;
    c.stats.v["pull_inspected"] += (double)h.pull_inspected;
    c.stats.v["pull_new"] += (double)h.pull_new;
    c.stats.v["launches"] += launched;
    c.stats.v["solves"] += 1.0;
    g.bfs_levels_hint.store(h.level, std::memory_order_relaxed);
}

}  // namespace gfr
