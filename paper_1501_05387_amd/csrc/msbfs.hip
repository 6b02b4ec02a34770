// msbfs.hip -- up to 64 BFS from different sources in one traversal
// (bitmask-packed multi-source BFS).  Each vertex carries 64-bit masks
// (bit q = source q): visited, current frontier and next frontier.  One read
// of a neighbour list serves every source whose frontier holds the vertex, so
// k sources cost about one traversal's worth of CSR traffic instead of k.
// The per-source results equal k single-source BFS (Sec. 5.1): a vertex gets
// depth L+1 for source q exactly when it is unvisited for q and has a
// neighbour in q's level-L frontier.
//
// Every level is three launches:
//   msbfs_level     advance.  Push: load-balanced edge chunks over the queue
//                   of frontier vertices (as in bfs.hip); an edge u->v adds
//                   fr[u] & ~vis[v] to nx[v] (one 64-bit atomicOr, issued only
//                   when it contributes new bits).  Pull (Sec. 4.5): a
//                   load-balanced sweep over all neighbour lists ORs the
//                   frontier masks of every vertex's neighbours, limited to
//                   the sources the vertex still needs; with many sources a
//                   vertex rarely finds all of them early, so the sweep is
//                   balanced over edges rather than cut short per vertex.
//   msbfs_finalize  lane = vertex: new = nx[v]; vis |= new; fr = new; the
//                   new mask is kept as the per-level record lvl[L+1][v]
//                   (one coalesced 8-byte store per vertex), and the vertex
//                   gets a mark byte if its mask is non-empty.  Past the
//                   record's capacity (and in serving sessions) the depths
//                   L+1 are written straight into the [k][n] output instead.
//   after the traversal, msbfs_output turns the level records into the
//   depth rows: every output line is written once and whole (writing each
//   level's depths into the rows left partial lines, level after level,
//   which ran at a fifth of the write bandwidth), and -1 goes where a source
//   never reached the vertex, so the output needs no fill.
//   compact         queue of the new frontier + level control (compact.h).
#include <algorithm>
#include <vector>

#include "compact.h"
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { MS_PUSH = 0, MS_PULL = 1, MS_DONE = 2 };

struct MsCtl {
    uint32_t dir;
    int32_t level;     // depth of the current frontier (-1 before the sources are placed)
    uint32_t nf, mf;
    uint32_t parity, err;
    float alpha;       // pull when frontier edges > m / alpha
    uint32_t pad;
    unsigned long long m;
    unsigned long long push_edges, pull_levels, push_levels;
    unsigned long long allq;     // sources (lanes) in use
    unsigned long long active;   // lanes whose frontier is non-empty after the last level
};

struct MsArgs {
    const int32_t *R;
    const int32_t *C;
    int32_t n;
    uint32_t nwords;
    unsigned long long *vis, *fr, *nx;
    uint8_t *mark;
    int32_t *depth;    // [k][n]
    int32_t k;
    unsigned long long *lvl;        // [lvl_cap][n] new-vertex masks per depth (null: write depths directly)
    int32_t lvl_cap;
    unsigned long long allq;
    const int32_t *base;            // [64] depth written = level + 1 - base[lane]
    unsigned long long *actp;       // [gridDim of finalize] per-group OR of the new frontier masks
    uint32_t nactp;
    FrontierQ q;
    FrontierQ full;            // every vertex with edges (pull sweeps)
    uint32_t full_nf, full_mf;
    MsCtl *ctl;
};

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void msbfs_level(MsArgs a)
{
    MsCtl *ctl = a.ctl;
    const uint32_t dir = ctl->dir;
    if (dir == MS_DONE || ctl->level < 0) return;
    // one LDS block serves both directions (28.7 KB at CH = 1024: five
    // work-groups per CU)
    __shared__ unsigned long long s_raw[2 * (CH + 1) + 3 * (CH + 2) / 2];
    if (dir == MS_PUSH) {
        unsigned long long *s_m = s_raw;
        uint32_t *s_off = (uint32_t *)(s_raw + (CH + 1));
        int32_t *s_row = (int32_t *)(s_off + (CH + 1));
        const uint32_t mf = ctl->mf, nf = ctl->nf;
        const FrontierQ q = a.q;
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
                s_m[i] = a.fr[q.v[s + i]];
            }
            __syncthreads();
            // each thread takes every GFR_BLOCK-th edge of the chunk; all its
            // column loads are issued first, then all mask loads (an edge past
            // the chunk end repeats the chunk's first edge and adds nothing)
            constexpr int PER = CH / GFR_BLOCK;
            int32_t vv[PER];
            unsigned long long mm[PER], vis[PER], nx[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const uint32_t e = e0 + p * GFR_BLOCK + threadIdx.x;
                const bool ok = e < e1;
                const uint32_t ec = ok ? e : e0;
                const int i = upper_index(s_off, 0, cnt - 1, ec);
                vv[p] = a.C[s_row[i] + (int32_t)(ec - s_off[i])];
                mm[p] = ok ? s_m[i] : 0ull;
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                vis[p] = a.vis[vv[p]];
                nx[p] = a.nx[vv[p]];
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const unsigned long long add = mm[p] & ~(vis[p] | nx[p]);
                if (add) atomicOr(a.nx + vv[p], add);
            }
        }
    } else {
        // pull: load-balanced sweep over every vertex's list (the whole-graph
        // queue), OR of the neighbours' frontier masks per vertex in LDS,
        // restricted to the sources the vertex still needs
        unsigned long long *s_need = s_raw, *s_acc = s_raw + (CH + 1);
        uint32_t *s_off = (uint32_t *)(s_raw + 2 * (CH + 1));
        int32_t *s_row = (int32_t *)(s_off + (CH + 1));
        int32_t *s_v = s_row + (CH + 1);
        const FrontierQ q = a.full;
        const uint32_t nf = a.full_nf, mf = a.full_mf;
        const unsigned long long allq = ctl->allq;
        const uint32_t nchunks = (mf + CH - 1) / CH;
        for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
            const uint32_t e0 = c * CH;
            const uint32_t e1 = min(e0 + (uint32_t)CH, mf);
            const int s = q.part[c];
            const int t = (c + 1 < nchunks) ? q.part[c + 1] : (int)nf - 1;
            const int cnt = t - s + 1;
            __syncthreads();
            for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
                const int32_t v = q.v[s + i];
                s_off[i] = q.off[s + i];
                s_row[i] = q.row[s + i];
                s_v[i] = v;
                s_need[i] = allq & ~a.vis[v];
                s_acc[i] = 0ull;
            }
            __syncthreads();
            // each thread takes every GFR_BLOCK-th edge of the chunk: the
            // column loads of the edges whose vertex still needs a source are
            // issued first, then their neighbours' mask loads, then the ORs
            constexpr int PER = CH / GFR_BLOCK;
            int ii[PER];
            int32_t uu[PER];
            unsigned long long ff[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const uint32_t k = p * GFR_BLOCK + threadIdx.x;
                const bool ok = k < e1 - e0;
                const uint32_t e = e0 + (ok ? k : 0u);
                ii[p] = upper_index(s_off, 0, cnt - 1, e);
                uu[p] = -1;
                if (ok && s_need[ii[p]]) uu[p] = a.C[s_row[ii[p]] + (int32_t)(e - s_off[ii[p]])];
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) ff[p] = uu[p] >= 0 ? a.fr[uu[p]] : 0ull;
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const unsigned long long f = ff[p] & s_need[ii[p]];
                if (f) atomicOr(s_acc + ii[p], f);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < cnt; i += GFR_BLOCK)
                if (s_acc[i]) atomicOr(a.nx + s_v[i], s_acc[i]);
        }
    }
}

// lane = vertex: fold the next-frontier masks into visited / frontier, write
// the level record (or depths L+1 row by row, 64 consecutive vertices per
// store), mark non-empty vertices for the compaction.
__global__ __launch_bounds__(GFR_BLOCK) void msbfs_finalize(MsArgs a)
{
    MsCtl *ctl = a.ctl;
    if (ctl->dir == MS_DONE) return;
    const int32_t L = ctl->level;
    const uint32_t waves = gridDim.x * GFR_WAVES;
    unsigned long long act = 0;   // lanes with a non-empty new frontier (wave-uniform)
    for (uint32_t grp = blockIdx.x * GFR_WAVES + threadIdx.x / 64; grp * 64u < (uint32_t)a.n; grp += waves) {
        const int32_t v = (int32_t)(grp * 64u) + lane_id();
        unsigned long long nw = 0;
        if (v < a.n) {
            nw = a.nx[v];
            const unsigned long long old = a.fr[v];
            if (nw) {
                a.nx[v] = 0ull;
                a.vis[v] |= nw;
                a.mark[v] = 1;
            }
            if (nw || old) a.fr[v] = nw;
        }
        // OR of the wave's masks -> the sources that need a row store
        unsigned long long any = nw;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)any, d, 64);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(any >> 32), d, 64);
            any |= ((unsigned long long)hi << 32) | lo;
        }
        act |= any;
        if (a.lvl && L + 1 < a.lvl_cap) {   // uniform: record the level, rows come later
            if (v < a.n) a.lvl[(size_t)(L + 1) * a.n + v] = nw;
            continue;
        }
        while (any) {
            const int qq = __ffsll(any) - 1;
            any &= any - 1;
            if ((nw >> qq) & 1ull) a.depth[(size_t)qq * a.n + v] = L + 1 - a.base[qq];
        }
    }
    __shared__ unsigned long long s_act[GFR_WAVES];
    if (lane_id() == 0) s_act[threadIdx.x / 64] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < GFR_WAVES; ++i) t |= s_act[i];
        a.actp[blockIdx.x] = t;
    }
}

// Depth rows from the level records of depths 0 .. nlev-1, lane = vertex.
// All records of the vertex are loaded first (clamped to the last valid one,
// then masked), folded into five bit planes (plane b = OR of the records
// whose depth has bit b set) and a found mask, so the depth of source q is
// read off bit q of the planes.  Then 64 coalesced row stores: -1 where the
// source never reached the vertex, the depth where a record holds it.
// Entries reached deeper than the records were written during the traversal
// and are left alone.
constexpr int32_t MS_LVL_CAP = 24;   // depths kept as records (5 bit planes cover them)
constexpr int32_t MS_DEEP = INT32_MIN;
static_assert(MS_LVL_CAP <= 32, "five bit planes hold depths below 32");

// The depths of vertex v for every source from its level records: bit b of
// plane[b] is bit b of the depth (a vertex is recorded at one depth per
// source).  -1 where the source never reached v; MS_DEEP marks a depth past
// the records, already written by msbfs_finalize.
__device__ __forceinline__ int32_t ms_depth_of(const unsigned long long *plane, unsigned long long found,
                                               unsigned long long vis, int q, int32_t base)
{
    int32_t d = 0;
#pragma unroll
    for (int bit = 0; bit < 5; ++bit) d |= (int32_t)((plane[bit] >> q) & 1ull) << bit;
    const bool rec_q = (found >> q) & 1ull, seen = (vis >> q) & 1ull;
    return rec_q ? d - base : (seen ? MS_DEEP : -1);
}

__global__ __launch_bounds__(GFR_BLOCK) void msbfs_output(MsArgs a)
{
    // depths 0 .. level were recorded (the last record is the empty frontier)
    const int32_t nlev = min(MS_LVL_CAP, a.ctl->level + 1);
    const int32_t kq = a.k;
    const size_t n = (size_t)a.n;
    if (n % 4 == 0 && ((uintptr_t)a.depth & 15) == 0) {
        // four consecutive vertices per thread: 32-byte record loads and one
        // 16-byte store per source row (every row then starts 16-byte aligned;
        // the records and masks are arena memory, 256-byte aligned)
        for (size_t v0 = ((size_t)blockIdx.x * GFR_BLOCK + threadIdx.x) * 4; v0 < n;
             v0 += (size_t)gridDim.x * GFR_BLOCK * 4) {
            unsigned long long plane[4][5], found[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                found[j] = 0;
#pragma unroll
                for (int bit = 0; bit < 5; ++bit) plane[j][bit] = 0;
            }
            for (int d = 0; d < nlev; ++d) {
                const ulonglong2 *r2 = (const ulonglong2 *)(a.lvl + (size_t)d * n + v0);
                const ulonglong2 lo = r2[0], hi = r2[1];
                const unsigned long long r[4] = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    found[j] |= r[j];
#pragma unroll
                    for (int bit = 0; bit < 5; ++bit)
                        if ((d >> bit) & 1) plane[j][bit] |= r[j];
                }
            }
            const ulonglong2 *vis2 = (const ulonglong2 *)(a.vis + v0);
            const ulonglong2 va = vis2[0], vb = vis2[1];
            const unsigned long long vis[4] = {va.x, va.y, vb.x, vb.y};
            for (int q = 0; q < kq; ++q) {
                const int32_t base = a.base[q];
                int32_t x[4];
                bool deep = false;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    x[j] = ms_depth_of(plane[j], found[j], vis[j], q, base);
                    deep |= x[j] == MS_DEEP;
                }
                int32_t *row = a.depth + (size_t)q * n + v0;
                if (!deep) {
                    *(int4 *)row = make_int4(x[0], x[1], x[2], x[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (x[j] != MS_DEEP) row[j] = x[j];
                }
            }
        }
        return;
    }
    for (size_t v = (size_t)blockIdx.x * GFR_BLOCK + threadIdx.x; v - threadIdx.x < n;
         v += (size_t)gridDim.x * GFR_BLOCK) {
        const bool ok = v < n;
        const size_t vc = ok ? v : n - 1;
        unsigned long long plane[5] = {0, 0, 0, 0, 0}, found = 0;
        for (int d = 0; d < nlev; ++d) {
            const unsigned long long r = a.lvl[(size_t)d * n + vc];
            found |= r;
#pragma unroll
            for (int bit = 0; bit < 5; ++bit)
                if ((d >> bit) & 1) plane[bit] |= r;
        }
        const unsigned long long vis = a.vis[vc];
        for (int q = 0; q < kq; ++q) {
            const int32_t x = ms_depth_of(plane, found, vis, q, a.base[q]);
            if (ok && x != MS_DEEP) a.depth[(size_t)q * n + v] = x;
        }
    }
}

struct MsMarks {
    MsArgs a;
    __device__ bool skip() const { return a.ctl->dir == MS_DONE; }
    __device__ uint32_t mask(uint32_t w) const
    {
        const uint32_t m = marks_to_mask(a.mark + 32ull * w);
        if (m) clear_marks(a.mark + 32ull * w);
        return m;
    }
    __device__ void partial(uint32_t) {}
    __device__ void control(uint32_t nf2, uint32_t mf2) const
    {
        // lanes still running: OR of the finalize groups' partials
        unsigned long long act = 0;
        for (uint32_t i = threadIdx.x; i < a.nactp; i += GFR_BLOCK) act |= a.actp[i];
        __shared__ unsigned long long s_or[GFR_WAVES];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)act, d, 64);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(act >> 32), d, 64);
            act |= ((unsigned long long)hi << 32) | lo;
        }
        if (lane_id() == 0) s_or[threadIdx.x / 64] = act;
        __syncthreads();
        if (threadIdx.x != 0) return;
        for (int i = 0; i < GFR_WAVES; ++i) act |= s_or[i];
        MsCtl *ctl = a.ctl;
        ctl->active = act;
        if (ctl->level >= 0) {
            if (ctl->dir == MS_PUSH) {
                ctl->push_levels += 1;
                ctl->push_edges += ctl->mf;
            } else {
                ctl->pull_levels += 1;
            }
        }
        uint32_t nd;
        if (nf2 == 0) nd = MS_DONE;
        else nd = ((double)mf2 > (double)ctl->m / ctl->alpha) ? MS_PULL : MS_PUSH;
        ctl->nf = nf2;
        ctl->mf = mf2;
        ctl->level += 1;
        ctl->parity ^= 1u;
        ctl->dir = nd;
    }
};

__global__ void msbfs_init(MsArgs a, const int32_t *src, float alpha)
{
    if (threadIdx.x == 0) {
        for (int32_t q = 0; q < a.k; ++q) a.nx[src[q]] |= 1ull << q;
        MsCtl *ctl = a.ctl;
        ctl->dir = MS_PUSH;
        ctl->level = -1;
        ctl->nf = ctl->mf = 0;
        ctl->parity = 0;
        ctl->err = 0;
        ctl->alpha = alpha;
        ctl->m = (unsigned long long)a.R[a.n];
        ctl->push_edges = ctl->pull_levels = ctl->push_levels = 0ull;
        ctl->allq = a.allq;
        ctl->active = 0ull;
    }
}

void run_bfs_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, int32_t *depth, hipStream_t s)
{
    const int32_t n = g.n;
    if (k < c.opt.batch_min_bfs) {   // a shared traversal costs about the same for few sources
        for (int32_t i = 0; i < k; ++i) run_bfs(c, g, sources[i], depth + (size_t)i * n, s);
        return;
    }
    const uint32_t chunk = 1024;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    const int G = grid_blocks(c, 5);   // the level kernel (28.7 KB of LDS) fits five work-groups per CU
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    // level records: 8 bytes per vertex and depth, for the first MS_LVL_CAP depths
    c.arena.reserve(3 * al256(8ull * n) + al256(32ull * nwords) + 3 * al256(4ull * n) + al256(4 * nparts) +
                    al256(16ull * cg.blocks) + al256(sizeof(MsCtl)) + 2 * al256(4 * 64) + al256(8ull * G) +
                    al256(8ull * n * MS_LVL_CAP));
    MsArgs a;
    memset(&a, 0, sizeof a);   // padding too: the bytes key the captured steps
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.n = n;
    a.nwords = nwords;
    a.full = g.full;
    a.full_nf = (uint32_t)g.full_nf;
    a.full_mf = (uint32_t)g.m;
    a.vis = c.arena.take<unsigned long long>(n);
    a.fr = c.arena.take<unsigned long long>(n);
    a.nx = c.arena.take<unsigned long long>(n);
    a.mark = c.arena.take<uint8_t>(32ull * nwords);
    a.q.v = c.arena.take<int32_t>(n);
    a.q.off = c.arena.take<uint32_t>(n);
    a.q.row = c.arena.take<int32_t>(n);
    a.q.part = c.arena.take<int32_t>(nparts);
    unsigned long long *status = c.arena.take<unsigned long long>(2ull * cg.blocks);
    a.ctl = c.arena.take<MsCtl>(1);
    int32_t *dsrc = c.arena.take<int32_t>(64);
    int32_t *base = c.arena.take<int32_t>(64);   // every source starts at level 0
    a.base = base;
    a.actp = c.arena.take<unsigned long long>(G);
    a.nactp = (uint32_t)G;
    a.lvl = c.arena.take<unsigned long long>((size_t)n * MS_LVL_CAP);
    a.lvl_cap = MS_LVL_CAP;
    fill_u32(base, 0u, 64, s);
    double levels = 0, pull_levels = 0, push_edges = 0;
    for (int32_t g0 = 0; g0 < k; g0 += 64) {
        const int32_t kk = std::min<int32_t>(64, k - g0);
        a.k = kk;
        a.allq = kk == 64 ? ~0ull : ((1ull << kk) - 1ull);
        a.depth = depth + (size_t)g0 * n;
        fill_u32(a.vis, 0u, 2ull * n, s);
        fill_u32(a.fr, 0u, 2ull * n, s);
        fill_u32(a.nx, 0u, 2ull * n, s);
        fill_u32(a.mark, 0u, 8ull * nwords, s);
        fill_u32(status, 0u, 4ull * cg.blocks, s);
        GFR_HIP(hipMemcpyAsync(dsrc, sources + g0, 4ull * kk, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(msbfs_init, dim3(1), dim3(64), 0, s, a, dsrc, (float)c.opt.msbfs_alpha);
        GFR_LAUNCH_CHECK();
        auto launch = [&]() {
            c.ktimer.run("msbfs_level", s, [&]() {
                hipLaunchKernelGGL(msbfs_level<GATHER_CH>, dim3(G), dim3(GFR_BLOCK), 0, s, a);
            });
            c.ktimer.run("msbfs_finalize", s, [&]() {
                hipLaunchKernelGGL(msbfs_finalize, dim3(G), dim3(GFR_BLOCK), 0, s, a);
            });
            c.ktimer.run("msbfs_compact", s, [&]() {
                hipLaunchKernelGGL(compact_kernel<MsMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, a.R, n, nwords,
                                   cg.wpt, MsMarks{a}, a.q, chunk, status, &a.ctl->parity, &a.ctl->err);
            });
        };
        StepKey key("msbfs");
        key.add(a).add(G).add(cg).add(chunk).add(status);
        run_until_done(c, &a.ctl->dir, MS_DONE, g.msbfs_levels_hint.load(std::memory_order_relaxed) + 2,
                       (int64_t)n + 8, s, launch, &key);
        // the output pass takes the depth count from the control block, so it
        // is queued before the block is read back (a failed batch fails the call)
        c.ktimer.run("msbfs_output", s, [&]() {
            hipLaunchKernelGGL(msbfs_output, dim3(grid_blocks(c, 8)), dim3(GFR_BLOCK), 0, s, a);
        });
        GFR_LAUNCH_CHECK();
        MsCtl h;
        GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(MsCtl), hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        memcpy(&h, c.pinned, sizeof(MsCtl));
        if (h.err) fail(GFR_E_DEVICE, "bfs_batch: frontier compaction look-back timed out");
        g.msbfs_levels_hint.store(h.level, std::memory_order_relaxed);
        levels += h.level;
        pull_levels += (double)h.pull_levels;
        push_edges += (double)h.push_edges;
    }
    c.stats.v["levels"] += levels;
    c.stats.v["pull_levels"] += pull_levels;
    c.stats.v["push_edges"] += push_edges;
    c.stats.v["solves"] += k;
}

// ---------------------------------------------------------------- sessions
// Lanes of a session join at a level boundary: their visited bits and depth
// row are cleared, the source enters the next frontier, and base[lane] makes
// depths count from the level it joined.  A lane whose new frontier is empty
// is finished; its depth row is final.

__global__ __launch_bounds__(GFR_BLOCK) void ms_clear_lanes(MsArgs a, unsigned long long lanes)
{
    const size_t n = (size_t)a.n;
    for (size_t v = (size_t)blockIdx.x * GFR_BLOCK + threadIdx.x; v < n; v += (size_t)gridDim.x * GFR_BLOCK) {
        a.vis[v] &= ~lanes;
        a.fr[v] &= ~lanes;
        a.nx[v] &= ~lanes;
        unsigned long long m = lanes;
        while (m) {
            const int q = __ffsll(m) - 1;
            m &= m - 1;
            a.depth[(size_t)q * n + v] = -1;
        }
    }
}

__global__ void ms_admit(MsArgs a, const int32_t *pairs, int32_t count, unsigned long long release)
{
    if (threadIdx.x != 0) return;
    MsCtl *ctl = a.ctl;
    unsigned long long allq = ctl->allq & ~release;
    for (int32_t i = 0; i < count; ++i) {
        const int32_t q = pairs[2 * i], src = pairs[2 * i + 1];
        a.nx[src] |= 1ull << q;
        ((int32_t *)a.base)[q] = ctl->level + 1;
        allq |= 1ull << q;
    }
    ctl->allq = allq;
    if (count && ctl->dir == MS_DONE) ctl->dir = MS_PUSH;
}

__global__ void ms_session_init(MsArgs a, float alpha)
{
    if (threadIdx.x != 0) return;
    MsCtl *ctl = a.ctl;
    ctl->dir = MS_DONE;
    ctl->level = -1;
    ctl->nf = ctl->mf = 0;
    ctl->parity = 0;
    ctl->err = 0;
    ctl->alpha = alpha;
    ctl->m = (unsigned long long)a.R[a.n];
    ctl->push_edges = ctl->pull_levels = ctl->push_levels = 0ull;
    ctl->allq = 0ull;
    ctl->active = 0ull;
}

namespace {
struct MsLayout {
    size_t n, nwords, nparts, G, blocks;
    size_t total() const
    {
        return 3 * al256(8 * n) + al256(32 * nwords) + 3 * al256(4 * n) + al256(4 * nparts) +
               al256(16 * blocks) + al256(sizeof(MsCtl)) + al256(4 * 64) + al256(8 * G) + al256(4 * 128) +
               al256(4 * 64 * n);
    }
};
MsLayout ms_layout(int64_t n, int64_t m, int num_cu)
{
    MsLayout L;
    L.n = (size_t)n;
    L.nwords = (size_t)((n + 63) / 64) * 2;
    L.nparts = (size_t)(m / 1024) + 2;
    L.G = (size_t)num_cu * 5;
    L.blocks = compact_geom((uint32_t)L.nwords, num_cu).blocks;
    return L;
}
}  // namespace

uint64_t bfs_session_bytes(int64_t n, int64_t m, int num_cu) { return ms_layout(n, m, num_cu).total(); }

struct MsSession final : LaneSession {
    Ctx &c;
    Graph &g;
    DevMem mem;
    MsArgs a{};
    CompactGeom cg{};
    int G = 0;
    uint32_t nwords = 0;
    unsigned long long *status = nullptr;
    int32_t *pairs = nullptr, *pin_pairs = nullptr;
    MsCtl *pin = nullptr;
    unsigned long long pending_release = 0;

    MsSession(Ctx &cc, Graph &gg, const Options &o) : c(cc), g(gg)
    {
        n = g.n;
        const MsLayout L = ms_layout(g.n, g.m, c.num_cu);
        nwords = (uint32_t)L.nwords;
        G = (int)L.G;
        cg = compact_geom(nwords, c.num_cu);
        bytes = L.total();
        GFR_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        GFR_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        GFR_HIP(hipHostMalloc((void **)&pin, sizeof(MsCtl), hipHostMallocDefault));
        GFR_HIP(hipHostMalloc((void **)&pin_pairs, 4 * 128, hipHostMallocDefault));
        mem.alloc(bytes);
        char *p = (char *)mem.p;
        auto take = [&](size_t b) {
            char *r = p;
            p += al256(b);
            return (void *)r;
        };
        a.R = g.R.as<int32_t>();
        a.C = g.C.as<int32_t>();
        a.n = g.n;
        a.nwords = nwords;
        a.full = g.full;
        a.full_nf = (uint32_t)g.full_nf;
        a.full_mf = (uint32_t)g.m;
        a.vis = (unsigned long long *)take(8 * L.n);
        a.fr = (unsigned long long *)take(8 * L.n);
        a.nx = (unsigned long long *)take(8 * L.n);
        a.mark = (uint8_t *)take(32 * L.nwords);
        a.q.v = (int32_t *)take(4 * L.n);
        a.q.off = (uint32_t *)take(4 * L.n);
        a.q.row = (int32_t *)take(4 * L.n);
        a.q.part = (int32_t *)take(4 * L.nparts);
        status = (unsigned long long *)take(16 * L.blocks);
        a.ctl = (MsCtl *)take(sizeof(MsCtl));
        a.base = (const int32_t *)take(4 * 64);
        a.actp = (unsigned long long *)take(8 * L.G);
        a.nactp = (uint32_t)G;
        pairs = (int32_t *)take(4 * 128);
        a.depth = (int32_t *)take(4 * 64 * L.n);
        a.k = 64;
        a.allq = 0;
        stage = a.depth;
        fill_u32(mem.p, 0u, (3 * al256(8 * L.n) + al256(32 * L.nwords)) / 4, stream);   // vis, fr, nx, marks
        fill_u32(status, 0u, 4 * L.blocks, stream);
        fill_u32((void *)a.base, 0u, 64, stream);
        hipLaunchKernelGGL(ms_session_init, dim3(1), dim3(64), 0, stream, a, (float)o.msbfs_alpha);
        GFR_LAUNCH_CHECK();
    }
    ~MsSession() override
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (pin) (void)hipHostFree(pin);
        if (pin_pairs) (void)hipHostFree(pin_pairs);
        if (done) (void)hipEventDestroy(done);
        if (stream) (void)hipStreamDestroy(stream);
    }
    void admit(const int32_t *lanes, const int32_t *sources, int32_t count) override
    {
        if (count <= 0) return;
        // the pinned staging of the previous admission must have been consumed
        GFR_HIP(hipStreamSynchronize(stream));
        unsigned long long mask = 0;
        for (int32_t i = 0; i < count; ++i) {
            pin_pairs[2 * i] = lanes[i];
            pin_pairs[2 * i + 1] = sources[i];
            mask |= 1ull << lanes[i];
        }
        GFR_HIP(hipMemcpyAsync(pairs, pin_pairs, 8ull * count, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(ms_clear_lanes, dim3(G), dim3(GFR_BLOCK), 0, stream, a, mask);
        hipLaunchKernelGGL(ms_admit, dim3(1), dim3(64), 0, stream, a, pairs, count, pending_release);
        GFR_LAUNCH_CHECK();
        pending_release = 0;
    }
    void release(unsigned long long lanes) override { pending_release |= lanes; }
    void pre_round() override
    {
        if (pending_release) {
            hipLaunchKernelGGL(ms_admit, dim3(1), dim3(64), 0, stream, a, pairs, 0, pending_release);
            pending_release = 0;
        }
    }
    void enqueue_step() override
    {
        hipLaunchKernelGGL(msbfs_level<GATHER_CH>, dim3(G), dim3(GFR_BLOCK), 0, stream, a);
        hipLaunchKernelGGL(msbfs_finalize, dim3(G), dim3(GFR_BLOCK), 0, stream, a);
        hipLaunchKernelGGL(compact_kernel<MsMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, stream, a.R, a.n, nwords,
                           cg.wpt, MsMarks{a}, a.q, 1024u, status, &a.ctl->parity, &a.ctl->err);
        GFR_LAUNCH_CHECK();
        GFR_HIP(hipMemcpyAsync(pin, a.ctl, sizeof(MsCtl), hipMemcpyDeviceToHost, stream));
    }
    // once the level loop has stopped, every lane's frontier is empty
    unsigned long long active() const override { return pin->dir == MS_DONE ? 0ull : pin->active; }
    gfr_status failed(std::string &msg) const override
    {
        if (pin->err) {
            msg = "bfs query: frontier compaction look-back timed out";
            return GFR_E_DEVICE;
        }
        return GFR_OK;
    }
    void extract(unsigned long long) override {}   // depth rows are written in place
};

std::unique_ptr<LaneSession> make_bfs_session(Ctx &c, Graph &g, const Options &o)
{
    return std::unique_ptr<LaneSession>(new MsSession(c, g, o));
}

}  // namespace gfr
