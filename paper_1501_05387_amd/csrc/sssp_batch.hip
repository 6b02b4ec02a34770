// sssp_batch.hip -- up to 64 SSSP queries in one traversal, lane = query.
//
// Distances are stored per vertex as a row of 64 uint32 (one per query, 256
// bytes).  A wave relaxes one edge u->v for all queries at once: lane q reads
// dist[u][q] and dist[v][q] inside two coalesced rows and applies the
// relaxation of Sec. 4.1 Algorithm 1 (atomicMin on improvement) only if u is
// in query q's frontier.  So a random access into the distance array costs
// one 256-byte row for up to 64 queries instead of one 64-byte line per
// query, and every CSR read is shared.  Each query's result equals its
// single-source SSSP; the queries share the near/far bucket bound of the
// priority queue (Sec. 4.5), which only changes the schedule, not the result.
//
// Narrow rows (an option; 32-bit rows are the default): a batch first runs
// with 8-bit distances (64-byte rows, a quarter of the bytes of every random
// row access), unreached = 0xFF.  A relaxation that would store 0xFF or more
// sets the overflow flag, the traversal stops, and the batch is solved again
// with 16-bit rows (128 bytes, unreached 0xFFFF), and past those with 32-bit
// rows; so a finished narrow batch stored exactly the distances the wide one
// would.  The 2 or 4 queries that share a 32-bit word of a narrow row lower
// it together with compare-and-swap (there is no 8- or 16-bit atomic
// minimum), which is why the narrow forms are slower on this GPU.
//
// Marks: per vertex a 64-bit mask of the queries improved in an iteration
// (one atomicOr of the wave's ballot per improved edge, not one byte store
// per improving lane) plus a byte any[v] for the compaction's scan.
//
// Pending queries: a queued vertex relaxes its queued queries and, read from
// its marks of the running launch, the queries improved at it earlier in the
// same launch (the marks stay; the vertex is queued for them again).  A
// relaxation with any distance a path has reached is safe, and carrying an
// improvement one launch early saves later launches the visits it would have
// caused (R-MAT s22, 64 queries: 4.03 m -> 3.74 m edge visits, 31.1 -> 30.0 ms).
//
// Sparse groups: a group of 64 edges whose edges each carry at most a few
// queries (option, default 8) is relaxed with lane = edge, one query per turn,
// loading 4-byte distances rather than 256-byte rows.  Such groups are most of
// the second launch (the sources' neighbours) and of the tail launches (R-MAT
// s22, 64 queries: 30.0 -> 28.0 ms per batch, the same visits).
//
// Every iteration is two launches:
//   bsssp_relax   load-balanced edge chunks over the near queue; each wave
//                 takes a quarter of the chunk, 64 edges at a time: lane l
//                 fetches edge l's target, weight, source and query mask
//                 (coalesced; the next group's fetch is issued before the
//                 current group relaxes), then the wave relaxes the 64 edges eight at a
//                 time with their sixteen distance rows in flight; a group
//                 whose 64 edges all leave one vertex loads that vertex's
//                 row once and relaxes sixteen edges at a time.
//   compact       near queue in vertex order with its per-vertex query masks,
//                 or, when the near queue has run dry, the far split with
//                 the next bucket (compact.h), plus the control.
#include <algorithm>
#include <type_traits>

#include "compact.h"
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { BS_RELAX = 0, BS_SPLIT = 1, BS_DONE = 2 };
enum : uint32_t { BS_PUSH = 0, BS_PULL = 1 };

struct BsCtl {
    uint32_t mode;
    uint32_t nf, mf;
    uint32_t iter;
    uint32_t lo, hi, delta;
    uint32_t far_any;
    uint32_t split_kept, split_min;
    uint32_t overflow, parity, err, splits;
    unsigned long long relaxed, improvements, pair_entries;
    unsigned long long active;   // queries with a (vertex, query) pair in the next near queue
    uint32_t dir;                // BS_PUSH / BS_PULL for the next relaxation
    float pull_alpha;            // pull when the frontier's edges exceed m / pull_alpha (0: never)
    unsigned long long m;
    uint32_t pull_iters, pad2;
    unsigned long long lane_relaxed;   // (edge, query) relaxations: edges visited x queries active at the source
    uint32_t unfit;              // 32-bit rows: a relaxation's sum did not fit below 0xFFFFFFFF (checked after the batch)
    uint32_t pad3;
};

struct BsArgs {
    const int32_t *R;
    const int32_t *C;
    const uint32_t *W;
    int32_t n;
    uint32_t nwords;
    uint32_t *D;                 // [n][64] 32-bit rows
    uint16_t *D16;               // [n][64] 16-bit rows (the same memory)
    uint8_t *D8;                 // [n][64] 8-bit rows (the same memory)
    unsigned long long *qm;      // query mask of every queued vertex
    unsigned long long *nq, *fq; // [n] queries improved into the near / far set
    uint8_t *nany, *fany;        // [n] (padded)
    FrontierQ q;
    uint32_t *part;              // per work-group [improvements, far marks written, lane relaxations, 0]
    unsigned long long *actp;    // per compaction group: OR of the query masks it queued
    uint32_t *fbits;             // [nwords] frontier bitmap of the next relaxation (qm valid where set)
    uint32_t pending;            // a source also relaxes the queries improved at it earlier in the launch
    uint32_t sparse;             // a group of 64 edges with at most this many queries per edge is relaxed
                                 // lane = edge (32-bit rows; 0: never)
    FrontierQ full;              // every vertex with edges (pull sweeps)
    uint32_t full_nf, full_mf;
    BsCtl *ctl;
};

constexpr int BS_UNROLL = 8;   // edges relaxed together (two distance rows each)
constexpr uint32_t BS_INF = 0xFFFFFFFFu;
constexpr uint32_t BS_INF16 = 0xFFFFu;

// unreached value of a row of BITS-bit distances
template <int BITS> __device__ __forceinline__ constexpr uint32_t row_inf()
{
    return BITS == 8 ? 0xFFu : BITS == 16 ? 0xFFFFu : 0xFFFFFFFFu;
}

// distance of query q at vertex v in 32-bit form (unreached: BS_INF)
template <int BITS>
__device__ __forceinline__ uint32_t bs_load(const BsArgs &a, size_t v, int q)
{
    if (BITS == 8) {
        const uint32_t x = a.D8[v * 64 + q];
        return x == 0xFFu ? BS_INF : x;
    }
    if (BITS == 16) {
        const uint32_t x = a.D16[v * 64 + q];
        return x == BS_INF16 ? BS_INF : x;
    }
    return a.D[v * 64 + q];
}

template <int BITS>
__device__ __forceinline__ void bs_store(const BsArgs &a, size_t v, int q, uint32_t d)
{
    if (BITS == 8) a.D8[v * 64 + q] = (uint8_t)(d == BS_INF ? 0xFFu : d);
    else if (BITS == 16) a.D16[v * 64 + q] = (uint16_t)(d == BS_INF ? BS_INF16 : d);
    else a.D[v * 64 + q] = d;
}

// Lower the distance of the calling lane's query at vertex v to nd where
// `imp` is set; `cur` is the value the lane loaded.  Called by the whole
// wave.  32-bit rows: one non-returning atomicMin per improving lane.
// Narrow rows: the first lane of each group of 32 / BITS lanes writes the
// group's word by compare-and-swap (a failed swap returns a word another
// update lowered; the minima are taken again against it until the swap
// succeeds or nothing is left to lower).
template <int BITS>
__device__ __forceinline__ void bs_lower(const BsArgs &a, size_t v, int lane, uint32_t nd, bool imp, uint32_t cur)
{
    if (BITS == 32) {
        if (imp) atomicMin(a.D + v * 64 + lane, nd);
        return;
    }
    constexpr int PER = 32 / BITS;   // lanes per 32-bit word
    constexpr uint32_t INF = row_inf<BITS>();
    const uint32_t want = imp ? nd : INF;   // nd < INF wherever imp holds
    const uint32_t raw = cur == BS_INF ? INF : cur;
    const int base = lane & ~(PER - 1);
    uint32_t wv[PER], rv[PER];
    bool lower = false;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        wv[j] = (uint32_t)__shfl((int)want, base + j, 64);
        rv[j] = (uint32_t)__shfl((int)raw, base + j, 64);
        lower |= wv[j] < rv[j];
    }
    if (lane == base && lower) {
        uint32_t *w = (uint32_t *)(a.D8 + (v * 64 + lane) * (BITS / 8));
        uint32_t expect = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) expect |= rv[j] << (BITS * j);
        for (;;) {
            uint32_t desired = 0;
#pragma unroll
            for (int j = 0; j < PER; ++j) desired |= min((expect >> (BITS * j)) & INF, wv[j]) << (BITS * j);
            if (desired == expect) break;
            const uint32_t old = atomicCAS(w, expect, desired);
            if (old == expect) break;
            expect = old;
        }
    }
}

__device__ __forceinline__ int32_t lane_bcast(int32_t x, int j) { return __builtin_amdgcn_readlane(x, j); }

template <int CH, int BITS>
__global__ __launch_bounds__(GFR_BLOCK) void bsssp_relax(BsArgs a)
{
    BsCtl *ctl = a.ctl;
    if (ctl->mode != BS_RELAX || ctl->dir != BS_PUSH) return;
    const uint32_t hi = ctl->hi, nf = ctl->nf, mf = ctl->mf;
    const FrontierQ q = a.q;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    constexpr uint32_t QW = CH / GFR_WAVES;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    uint32_t nimp = 0, nfar = 0, nlr = 0;
    bool ovf = false, unf = false;
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
        const uint32_t eb = e0 + wave * QW, ee = min(eb + QW, e1);
        if (eb >= ee) continue;
        int ilo = upper_index(s_off, 0, cnt - 1, eb);
        // lane l of a group describes edge e + l (target, weight, source, query
        // mask); the next group's loads are issued before this group relaxes
        auto fetch = [&](uint32_t e, int nbx, int32_t &vx, int32_t &wx, int32_t &ux, unsigned long long &qx) {
            const uint32_t el = e + (uint32_t)min(lane, nbx - 1);
            const int il = upper_index(s_off, ilo, min(cnt - 1, ilo + lane + 1), el);
            const int32_t idx = s_row[il] + (int32_t)(el - s_off[il]);
            vx = a.C[idx];
            wx = (int32_t)a.W[idx];
            ux = s_v[il];
            qx = a.qm[ux];
            if (a.pending) qx |= a.nq[ux];
            ilo = lane_bcast(il, nbx - 1);
        };
        int nbn = (int)min(64u, ee - eb);
        int32_t vn, wn, un;
        unsigned long long qn;
        fetch(eb, nbn, vn, wn, un, qn);
        for (uint32_t e = eb; e < ee; e += 64) {
            const int nb = nbn;
            const int32_t vl = vn, wl = wn, ul = un;
            const unsigned long long ql = qn;
            if (e + 64 < ee) {
                nbn = (int)min(64u, ee - (e + 64));
                fetch(e + 64, nbn, vn, wn, un, qn);
            }
            if (BITS == 32 && a.sparse != 0u && !ballot(lane < nb && (uint32_t)__popcll(ql) > a.sparse)) {
                // few queries per edge: lane l relaxes edge l for each of its
                // queries in turn, loading single 4-byte distances instead
                // of whole 256-byte rows (the turns that read words of one
                // row find its lines in cache after the first)
                unsigned long long rem = lane < nb ? ql : 0ull;
                while (ballot(rem != 0ull)) {
                    const bool has = rem != 0ull;
                    const int qq = has ? __ffsll(rem) - 1 : 0;
                    rem &= rem - 1ull;
                    const uint32_t du = has ? a.D[(size_t)ul * 64 + qq] : BS_INF;
                    const uint32_t dv = has ? a.D[(size_t)vl * 64 + qq] : 0u;
                    // as in the row form: a pending query whose distance has
                    // not arrived is skipped and keeps its mark
                    const bool act = has & (du != BS_INF);
                    const unsigned long long nd64 = (unsigned long long)du + (uint32_t)wl;
                    const bool fits = nd64 < 0xFFFFFFFFull;
                    const uint32_t nd = (uint32_t)nd64;
                    const bool imp = act & fits & (nd < dv);
                    unf |= act & !fits;
                    nlr += act ? 1u : 0u;
                    nimp += imp ? 1u : 0u;
                    if (imp) {
                        atomicMin(a.D + (size_t)vl * 64 + qq, nd);
                        if (nd < hi) {
                            atomicOr(a.nq + vl, 1ull << qq);
                            a.nany[vl] = 1;
                        } else {
                            atomicOr(a.fq + vl, 1ull << qq);
                            a.fany[vl] = 1;
                        }
                    }
                    if (ballot(imp & (nd >= hi)) != 0ull && lane == 0) ++nfar;
                }
                continue;
            }
            const int32_t qlo = (int32_t)(uint32_t)ql, qhi = (int32_t)(uint32_t)(ql >> 32);
            // one relaxation of edge (u, v, w) for this lane's query; the test
            // is computed for every lane, so that no load is moved into a
            // branch and waited for there
            auto relax = [&](int32_t v, uint32_t w, uint32_t du, uint32_t dv, bool act) {
                const unsigned long long nd64 = (unsigned long long)du + w;
                const bool fits = nd64 < 0xFFFFFFFFull;
                const uint32_t nd = (uint32_t)nd64;
                bool imp;
                if (BITS < 32) {
                    // an improvement that does not fit a narrow row stops the
                    // batch (it is solved again with wider rows), and so does
                    // a sum the 32-bit rows would reject
                    const bool cand = act & (nd64 < (unsigned long long)dv);
                    imp = cand & (nd64 < (unsigned long long)row_inf<BITS>());
                    ovf |= (cand & !imp) | (act & !fits);
                } else {
                    imp = act & fits & (nd < dv);
                    unf |= act & !fits;
                }
                nlr += act ? 1u : 0u;
                // the update does not return a value: the mark follows the
                // pre-check, a superset of the true improvements (a marked
                // vertex is simply relaxed again with its current distance)
                const bool near_imp = imp & (nd < hi), far_imp = imp & (nd >= hi);
                if (ballot(imp)) bs_lower<BITS>(a, (size_t)v, lane, nd, imp, dv);
                nimp += imp ? 1u : 0u;
                const uint64_t bn = ballot(near_imp), bf = ballot(far_imp);
                if (lane == 0) {
                    if (bn) {
                        atomicOr(a.nq + v, (unsigned long long)bn);
                        a.nany[v] = 1;
                    }
                    if (bf) {
                        atomicOr(a.fq + v, (unsigned long long)bf);
                        a.fany[v] = 1;
                        ++nfar;
                    }
                }
            };
            const int32_t u_first = lane_bcast(ul, 0);
            if (u_first == lane_bcast(ul, nb - 1)) {
                // the whole group leaves one vertex (edges are in source
                // order): its distance row and query bit are loaded once
                const uint32_t du = bs_load<BITS>(a, (size_t)u_first, lane);
                const uint32_t q0 = (uint32_t)lane_bcast(qlo, 0), q1 = (uint32_t)lane_bcast(qhi, 0);
                // a pending query read before its distance arrived here is not
                // relaxed (its mark stays, it is relaxed in a later launch)
                const bool act_u = ((((lane < 32 ? q0 : q1) >> (lane & 31)) & 1u) != 0) & (du != BS_INF);
                for (int j0 = 0; j0 < nb; j0 += 16) {
                    uint32_t dv[16], ww[16];
                    int32_t vv[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int src = min(j0 + j, nb - 1);   // a padded edge repeats the last one
                        vv[j] = lane_bcast(vl, src);
                        ww[j] = (uint32_t)lane_bcast(wl, src);
                        dv[j] = bs_load<BITS>(a, (size_t)vv[j], lane);
                    }
#pragma unroll
                    for (int j = 0; j < 16; ++j) relax(vv[j], ww[j], du, dv[j], act_u & (j0 + j < nb));
                }
            } else {
                // edges are in source order: a source row is loaded once per
                // run of edges that share it (about 5 sources per such group)
                int32_t uprev = -1;
                uint32_t duprev = 0;
                for (int j0 = 0; j0 < nb; j0 += BS_UNROLL) {
                    uint32_t du[BS_UNROLL], dv[BS_UNROLL], ww[BS_UNROLL], qw[BS_UNROLL];
                    int32_t vv[BS_UNROLL], uu[BS_UNROLL];
                    bool same[BS_UNROLL];
#pragma unroll
                    for (int j = 0; j < BS_UNROLL; ++j) {
                        const int src = min(j0 + j, nb - 1);
                        uu[j] = lane_bcast(ul, src);
                        same[j] = uu[j] == (j == 0 ? uprev : uu[j - 1]);   // wave-uniform
                        vv[j] = lane_bcast(vl, src);
                        ww[j] = (uint32_t)lane_bcast(wl, src);
                        const uint32_t q0 = (uint32_t)lane_bcast(qlo, src), q1 = (uint32_t)lane_bcast(qhi, src);
                        qw[j] = lane < 32 ? q0 : q1;
                        du[j] = 0u;
                        if (!same[j]) du[j] = bs_load<BITS>(a, (size_t)uu[j], lane);
                        dv[j] = bs_load<BITS>(a, (size_t)vv[j], lane);
                    }
#pragma unroll
                    for (int j = 0; j < BS_UNROLL; ++j)
                        if (same[j]) du[j] = j == 0 ? duprev : du[j - 1];
                    uprev = uu[BS_UNROLL - 1];
                    duprev = du[BS_UNROLL - 1];
#pragma unroll
                    for (int j = 0; j < BS_UNROLL; ++j)
                        relax(vv[j], ww[j], du[j], dv[j],
                              (j0 + j < nb) & (((qw[j] >> (lane & 31)) & 1u) != 0) & (du[j] != BS_INF));
                }
            }
        }
    }
    if (ovf) ctl->overflow = 1u;
    if (unf) ctl->unfit = 1u;
    __shared__ uint32_t s_a[GFR_WAVES], s_b[GFR_WAVES], s_c[GFR_WAVES];
    nimp = wave_sum_u32(nimp);
    nlr = wave_sum_u32(nlr);
    if (lane == 0) {
        s_a[wave] = nimp;
        s_b[wave] = nfar;
        s_c[wave] = nlr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0, y = 0, z = 0;
        for (int k = 0; k < GFR_WAVES; ++k) {
            x += s_a[k];
            y += s_b[k];
            z += s_c[k];
        }
        a.part[4 * blockIdx.x] = x;
        a.part[4 * blockIdx.x + 1] = y;
        a.part[4 * blockIdx.x + 2] = z;
    }
}

// bit i of x moved to bit 2i (a 32-bit value spread over 64 bits)
__device__ __forceinline__ unsigned long long spread2(uint32_t x32)
{
    unsigned long long x = x32;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// The relaxation of bsssp_relax with 32-bit rows, two edges per distance-row
// instruction: lanes 0-31 take edge A and lanes 32-63 edge B, lane k of a half
// holding queries 2k and 2k+1 of the row as one 8-byte word.  A random row
// costs about the same per instruction whatever its width, so this halves the
// row instructions of every edge visit.  Improving queries are lowered with
// non-returning atomicMin, as in bsssp_relax.
constexpr int BP2_U = 4;    // edge pairs relaxed together (source and target rows of each)
constexpr int BP2_UH = 8;   // edge pairs relaxed together when the group leaves one vertex

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void bsssp_relax2(BsArgs a)
{
    BsCtl *ctl = a.ctl;
    if (ctl->mode != BS_RELAX || ctl->dir != BS_PUSH) return;
    const uint32_t hi = ctl->hi, nf = ctl->nf, mf = ctl->mf;
    const FrontierQ q = a.q;
    const uint2 *D2 = (const uint2 *)a.D;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int half = lane >> 5, k = lane & 31;
    const int qshift = (2 * k) & 31;
    constexpr uint32_t QW = CH / GFR_WAVES;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    uint32_t nimp = 0, nfar = 0, nlr = 0;
    bool unf = false;
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
        const uint32_t eb = e0 + wave * QW, ee = min(eb + QW, e1);
        if (eb >= ee) continue;
        int ilo = upper_index(s_off, 0, cnt - 1, eb);
        auto fetch = [&](uint32_t e, int nbx, int32_t &vx, int32_t &wx, int32_t &ux, unsigned long long &qx) {
            const uint32_t el = e + (uint32_t)min(lane, nbx - 1);
            const int il = upper_index(s_off, ilo, min(cnt - 1, ilo + lane + 1), el);
            const int32_t idx = s_row[il] + (int32_t)(el - s_off[il]);
            vx = a.C[idx];
            wx = (int32_t)a.W[idx];
            ux = s_v[il];
            qx = a.qm[ux];
            ilo = lane_bcast(il, nbx - 1);
        };
        int nbn = (int)min(64u, ee - eb);
        int32_t vn, wn, un;
        unsigned long long qn;
        fetch(eb, nbn, vn, wn, un, qn);
        for (uint32_t e = eb; e < ee; e += 64) {
            const int nb = nbn;
            const int32_t vl = vn, wl = wn, ul = un;
            const unsigned long long ql = qn;
            if (e + 64 < ee) {
                nbn = (int)min(64u, ee - (e + 64));
                fetch(e + 64, nbn, vn, wn, un, qn);
            }
            const int32_t qlo = (int32_t)(uint32_t)ql, qhi = (int32_t)(uint32_t)(ql >> 32);
            // this lane's two query bits of the source of group edge j
            auto qbits = [&](int j) -> uint32_t {
                const uint32_t w = (uint32_t)(k < 16 ? lane_bcast(qlo, j) : lane_bcast(qhi, j));
                return (w >> qshift) & 3u;
            };
            // relax one edge pair: this lane's half holds edge j (targets vA / vB of the pair)
            auto relax2 = [&](int32_t vA, int32_t vB, int32_t v, uint32_t w, uint2 du, uint2 dv, uint32_t act) {
                const unsigned long long s0 = (unsigned long long)du.x + w, s1 = (unsigned long long)du.y + w;
                const bool a0 = act & 1u, a1 = (act >> 1) & 1u;
                const bool f0 = s0 < 0xFFFFFFFFull, f1 = s1 < 0xFFFFFFFFull;
                const uint32_t n0 = (uint32_t)s0, n1 = (uint32_t)s1;
                const bool i0 = a0 & f0 & (n0 < dv.x), i1 = a1 & f1 & (n1 < dv.y);
                unf |= (a0 & !f0) | (a1 & !f1);
                nlr += (a0 ? 1u : 0u) + (a1 ? 1u : 0u);
                nimp += (i0 ? 1u : 0u) + (i1 ? 1u : 0u);
                if (ballot(i0 | i1)) {
                    // non-returning updates; the marks follow the pre-check
                    uint32_t *row = a.D + (size_t)v * 64 + 2 * k;
                    if (i0) atomicMin(row, n0);
                    if (i1) atomicMin(row + 1, n1);
                    const uint64_t bn0 = ballot(i0 & (n0 < hi)), bn1 = ballot(i1 & (n1 < hi));
                    const uint64_t bf0 = ballot(i0 & (n0 >= hi)), bf1 = ballot(i1 & (n1 >= hi));
                    if (lane == 0) {
                        const unsigned long long nA = spread2((uint32_t)bn0) | (spread2((uint32_t)bn1) << 1);
                        const unsigned long long nB = spread2((uint32_t)(bn0 >> 32)) | (spread2((uint32_t)(bn1 >> 32)) << 1);
                        const unsigned long long fA = spread2((uint32_t)bf0) | (spread2((uint32_t)bf1) << 1);
                        const unsigned long long fB = spread2((uint32_t)(bf0 >> 32)) | (spread2((uint32_t)(bf1 >> 32)) << 1);
                        if (nA) {
                            atomicOr(a.nq + vA, nA);
                            a.nany[vA] = 1;
                        }
                        if (nB) {
                            atomicOr(a.nq + vB, nB);
                            a.nany[vB] = 1;
                        }
                        if (fA) {
                            atomicOr(a.fq + vA, fA);
                            a.fany[vA] = 1;
                            ++nfar;
                        }
                        if (fB) {
                            atomicOr(a.fq + vB, fB);
                            a.fany[vB] = 1;
                            ++nfar;
                        }
                    }
                }
            };
            const int32_t u_first = lane_bcast(ul, 0);
            if (u_first == lane_bcast(ul, nb - 1)) {
                // the whole group leaves one vertex: its row and query bits are loaded once
                const uint2 du = D2[(size_t)u_first * 32 + k];
                const uint32_t qb = qbits(0);
                for (int j0 = 0; j0 < nb; j0 += 2 * BP2_UH) {
                    uint2 dv[BP2_UH];
                    int32_t vv[BP2_UH], vA[BP2_UH], vB[BP2_UH];
                    uint32_t ww[BP2_UH];
#pragma unroll
                    for (int t2 = 0; t2 < BP2_UH; ++t2) {
                        const int jA = min(j0 + 2 * t2, nb - 1), jB = min(j0 + 2 * t2 + 1, nb - 1);
                        vA[t2] = lane_bcast(vl, jA);
                        vB[t2] = lane_bcast(vl, jB);
                        vv[t2] = half ? vB[t2] : vA[t2];
                        ww[t2] = (uint32_t)(half ? lane_bcast(wl, jB) : lane_bcast(wl, jA));
                        dv[t2] = D2[(size_t)vv[t2] * 32 + k];
                    }
#pragma unroll
                    for (int t2 = 0; t2 < BP2_UH; ++t2)
                        relax2(vA[t2], vB[t2], vv[t2], ww[t2], du, dv[t2], (j0 + 2 * t2 + half < nb) ? qb : 0u);
                }
            } else {
                for (int j0 = 0; j0 < nb; j0 += 2 * BP2_U) {
                    uint2 du[BP2_U], dv[BP2_U];
                    int32_t vv[BP2_U], vA[BP2_U], vB[BP2_U];
                    uint32_t ww[BP2_U], qb[BP2_U];
#pragma unroll
                    for (int t2 = 0; t2 < BP2_U; ++t2) {
                        const int jA = min(j0 + 2 * t2, nb - 1), jB = min(j0 + 2 * t2 + 1, nb - 1);
                        const int j = half ? jB : jA;
                        const int32_t uA = lane_bcast(ul, jA), uB = lane_bcast(ul, jB);
                        vA[t2] = lane_bcast(vl, jA);
                        vB[t2] = lane_bcast(vl, jB);
                        vv[t2] = half ? vB[t2] : vA[t2];
                        ww[t2] = (uint32_t)(half ? lane_bcast(wl, jB) : lane_bcast(wl, jA));
                        const uint32_t bA = qbits(jA), bB = qbits(jB);
                        qb[t2] = (j0 + 2 * t2 + half < nb) ? (half ? bB : bA) : 0u;
                        (void)j;
                        du[t2] = D2[(size_t)(half ? uB : uA) * 32 + k];
                        dv[t2] = D2[(size_t)vv[t2] * 32 + k];
                    }
#pragma unroll
                    for (int t2 = 0; t2 < BP2_U; ++t2) relax2(vA[t2], vB[t2], vv[t2], ww[t2], du[t2], dv[t2], qb[t2]);
                }
            }
        }
    }
    if (unf) ctl->unfit = 1u;
    __shared__ uint32_t s_a[GFR_WAVES], s_b[GFR_WAVES], s_c[GFR_WAVES];
    nimp = wave_sum_u32(nimp);
    nlr = wave_sum_u32(nlr);
    if (lane == 0) {
        s_a[wave] = nimp;
        s_b[wave] = nfar;
        s_c[wave] = nlr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0, y = 0, z = 0;
        for (int i = 0; i < GFR_WAVES; ++i) {
            x += s_a[i];
            y += s_b[i];
            z += s_c[i];
        }
        a.part[4 * blockIdx.x] = x;
        a.part[4 * blockIdx.x + 1] = y;
        a.part[4 * blockIdx.x + 2] = z;
    }
}

// Pull relaxation for frontiers that carry most of the edges: a
// load-balanced sweep over every vertex's list (the whole-graph queue).  An
// edge u->v with u in the frontier contributes dist[u][q] + w to a running
// minimum of v, per query q active at u; each wave flushes the minimum of an
// owner v once (one pre-checked atomicMin and mark per query) instead of once
// per improving edge.  Sources outside the frontier cost one bitmap probe.
constexpr int BP_UNROLL = 8;

template <int CH, int BITS>
__global__ __launch_bounds__(GFR_BLOCK) void bsssp_pull(BsArgs a)
{
    BsCtl *ctl = a.ctl;
    if (ctl->mode != BS_RELAX || ctl->dir != BS_PULL) return;
    const uint32_t hi = ctl->hi;
    const FrontierQ q = a.full;
    const uint32_t nf = a.full_nf, mf = a.full_mf;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    constexpr uint32_t QW = CH / GFR_WAVES;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    uint32_t nimp = 0, nfar = 0, nlr = 0;
    bool ovf = false, unf = false;
    int32_t cur = -1;                 // owner whose minimum is being formed (wave-uniform)
    uint32_t acc = 0xFFFFFFFFu;       // its minimum for this lane's query
    uint32_t old = 0;                 // the owner's distance, loaded when the owner starts
    auto flush = [&]() {
        if (cur >= 0) {
            bool imp = acc < old;
            if (BITS < 32 && imp && acc >= row_inf<BITS>()) {
                ovf = true;   // does not fit a narrow row: the batch is solved again with wider rows
                imp = false;
            }
            const bool near_imp = imp & (acc < hi), far_imp = imp & (acc >= hi);
            if (ballot(imp)) bs_lower<BITS>(a, (size_t)cur, lane, acc, imp, old);
            nimp += imp ? 1u : 0u;
            const uint64_t bn = ballot(near_imp), bf = ballot(far_imp);
            if (lane == 0) {
                if (bn) {
                    atomicOr(a.nq + cur, (unsigned long long)bn);
                    a.nany[cur] = 1;
                }
                if (bf) {
                    atomicOr(a.fq + cur, (unsigned long long)bf);
                    a.fany[cur] = 1;
                    ++nfar;
                }
            }
        }
        acc = 0xFFFFFFFFu;
    };
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
        const uint32_t eb = e0 + wave * QW, ee = min(eb + QW, e1);
        if (eb >= ee) continue;
        int ilo = upper_index(s_off, 0, cnt - 1, eb);
        for (uint32_t e = eb; e < ee; e += 64) {
            // lane l: edge e + l, its source u (the neighbour), owner v and,
            // if u is in the frontier, u's query mask (entry bounds as in
            // bsssp_relax)
            const int nb = (int)min(64u, ee - e);
            int32_t ul = 0, vl = 0, wl = 0, il = ilo;
            unsigned long long ql = 0;
            if (lane < nb) {
                const uint32_t el = e + lane;
                il = upper_index(s_off, ilo, min(cnt - 1, ilo + lane + 1), el);
                const int32_t idx = s_row[il] + (int32_t)(el - s_off[il]);
                ul = a.C[idx];
                wl = (int32_t)a.W[idx];
                vl = s_v[il];
                if ((a.fbits[ul >> 5] >> (ul & 31)) & 1u) ql = a.qm[ul];
            }
            ilo = lane_bcast(il, nb - 1);
            unsigned long long act = ballot(ql != 0ull);
            const int32_t qlo = (int32_t)(uint32_t)ql, qhi = (int32_t)(uint32_t)(ql >> 32);
            while (act) {
                // the next BP_UNROLL edges with a frontier source, in order;
                // their source rows are loaded together
                int jj[BP_UNROLL];
#pragma unroll
                for (int k = 0; k < BP_UNROLL; ++k) {
                    jj[k] = act ? __ffsll(act) - 1 : -1;
                    act &= act - 1;
                }
                uint32_t du[BP_UNROLL], ww[BP_UNROLL], qw[BP_UNROLL];
                int32_t vv[BP_UNROLL];
#pragma unroll
                for (int k = 0; k < BP_UNROLL; ++k) {
                    const int j = jj[k] < 0 ? jj[0] : jj[k];
                    const int32_t u = lane_bcast(ul, j);
                    vv[k] = lane_bcast(vl, j);
                    ww[k] = (uint32_t)lane_bcast(wl, j);
                    const uint32_t q0 = (uint32_t)lane_bcast(qlo, j), q1 = (uint32_t)lane_bcast(qhi, j);
                    qw[k] = lane < 32 ? q0 : q1;
                    du[k] = bs_load<BITS>(a, (size_t)u, lane);
                }
#pragma unroll
                for (int k = 0; k < BP_UNROLL; ++k) {
                    if (jj[k] < 0) break;
                    if (vv[k] != cur) {
                        flush();
                        cur = vv[k];
                        old = bs_load<BITS>(a, (size_t)cur, lane);   // read by the owner's flush
                    }
                    const bool on = ((qw[k] >> (lane & 31)) & 1u) != 0;
                    nlr += on ? 1u : 0u;
                    const unsigned long long nd64 = (unsigned long long)du[k] + ww[k];
                    const bool fits = nd64 < 0xFFFFFFFFull;
                    // a narrow batch is solved again with wider rows; 32-bit rows note it for the final check
                    if (BITS < 32) ovf |= on & !fits;
                    else unf |= on & !fits;
                    const uint32_t nd = (uint32_t)nd64;
                    acc = (on & fits & (nd < acc)) ? nd : acc;
                }
            }
        }
        flush();
        cur = -1;
    }
    if (ovf) ctl->overflow = 1u;
    if (unf) ctl->unfit = 1u;
    __shared__ uint32_t s_a[GFR_WAVES], s_b[GFR_WAVES], s_c[GFR_WAVES];
    nimp = wave_sum_u32(nimp);
    nlr = wave_sum_u32(nlr);
    if (lane == 0) {
        s_a[wave] = nimp;
        s_b[wave] = nfar;
        s_c[wave] = nlr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0, y = 0, z = 0;
        for (int k = 0; k < GFR_WAVES; ++k) {
            x += s_a[k];
            y += s_b[k];
            z += s_c[k];
        }
        a.part[4 * blockIdx.x] = x;
        a.part[4 * blockIdx.x + 1] = y;
        a.part[4 * blockIdx.x + 2] = z;
    }
}

// 64 mark bytes (0/1) of one vertex -> query mask; clears them when `clear`
template <int BITS>
struct BsMarks {
    BsArgs a;
    uint32_t nparts;
    uint32_t nactp;   // compaction groups
    uint32_t wave_run = 0;   // every thread owns one word: a wave's 64 words are consecutive
    uint32_t kept = 0, kmin = 0xFFFFFFFFu;
    unsigned long long actq = 0;
    uint32_t pairs = 0;   // (vertex, query) pairs queued by this thread

    __device__ bool skip() const { return a.ctl->mode == BS_DONE; }

    __device__ uint32_t mask(uint32_t w)
    {
        BsCtl *ctl = a.ctl;
        if (ctl->mode == BS_RELAX) {
            const uint32_t m = marks_to_mask(a.nany + 32ull * w);
            a.fbits[w] = m;
            if (wave_run && ballot(true) == ~0ull) {
                // a dense run of 64 words (at least 8 marked vertices a word on
                // average, all 2048 vertices below n): the wave moves their
                // masks as one coalesced 16 KB block, lane l taking 16-byte
                // pieces l, l + 64, ... (a vertex without the mark has a zero
                // mask, and its qm is never read)
                const uint32_t wfirst = (uint32_t)__builtin_amdgcn_readfirstlane((int)w);
                const uint32_t tot = wave_sum_u32(__popc(m));
                if (tot >= 64u * 8u && (wfirst + 64ull) * 32ull <= (unsigned long long)a.n) {
                    if (m) clear_marks(a.nany + 32ull * w);
                    ulonglong2 *pn = (ulonglong2 *)(a.nq + 32ull * wfirst);
                    ulonglong2 *pq = (ulonglong2 *)(a.qm + 32ull * wfirst);
                    const int l = lane_id();
                    ulonglong2 x[16];
#pragma unroll
                    for (int it = 0; it < 16; ++it) x[it] = pn[it * 64 + l];
#pragma unroll
                    for (int it = 0; it < 16; ++it) {
                        pn[it * 64 + l] = make_ulonglong2(0ull, 0ull);
                        pq[it * 64 + l] = x[it];
                        actq |= x[it].x | x[it].y;
                        pairs += __popcll(x[it].x) + __popcll(x[it].y);
                    }
                    return m;
                }
            }
            if (!m) return 0u;
            clear_marks(a.nany + 32ull * w);
            if (__popc(m) >= 8) {
                // a dense word: its 32 masks move as 256 contiguous bytes (a vertex
                // without the mark has a zero mask, and its qm is never read)
                ulonglong2 *pn = (ulonglong2 *)(a.nq + 32ull * w);
                ulonglong2 *pq = (ulonglong2 *)(a.qm + 32ull * w);
                ulonglong2 x[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) x[i] = pn[i];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    pn[i] = make_ulonglong2(0ull, 0ull);
                    pq[i] = x[i];
                    actq |= x[i].x | x[i].y;
                    pairs += __popcll(x[i].x) + __popcll(x[i].y);
                }
                return m;
            }
            uint32_t bits = m;
            while (bits) {
                const int bi = __ffs(bits) - 1;
                bits &= bits - 1;
                const uint32_t v = w * 32u + bi;
                const unsigned long long qv = a.nq[v];
                a.nq[v] = 0ull;
                a.qm[v] = qv;
                actq |= qv;
                pairs += __popcll(qv);
            }
            return m;
        }
        const uint32_t f = marks_to_mask(a.fany + 32ull * w);
        if (!f) {
            a.fbits[w] = 0u;
            return 0u;
        }
        const uint32_t lo = ctl->lo, hi = ctl->hi;
        uint32_t out = 0, bits = f;
        while (bits) {
            const int bi = __ffs(bits) - 1;
            bits &= bits - 1;
            const uint32_t v = w * 32u + bi;
            unsigned long long fm = a.fq[v], nm = 0, left = 0;
            while (fm) {
                const int qq = __ffsll(fm) - 1;
                fm &= fm - 1;
                const uint32_t d = bs_load<BITS>(a, (size_t)v, qq);
                if (d < hi) {
                    if (d >= lo) nm |= 1ull << qq;
                } else {
                    left |= 1ull << qq;
                    ++kept;
                    kmin = min(kmin, d);
                }
            }
            a.fq[v] = left;
            if (!left) a.fany[v] = 0;
            if (nm) {
                a.qm[v] = nm;
                out |= 1u << bi;
                pairs += __popcll(nm);
            }
        }
        a.fbits[w] = out;
        return out;
    }

    __device__ void partial(uint32_t)
    {
        {
            __shared__ uint32_t s_p[GFR_WAVES];
            const uint32_t p = wave_sum_u32(pairs);
            if (lane_id() == 0) s_p[threadIdx.x / 64] = p;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t t = 0;
                for (int i = 0; i < GFR_WAVES; ++i) t += s_p[i];
                if (t) atomicAdd(&a.ctl->pair_entries, (unsigned long long)t);
            }
        }
        if (a.ctl->mode == BS_RELAX) {
            // OR of the queued query masks of this group
            __shared__ unsigned long long s_q[GFR_WAVES];
            unsigned long long x = actq;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, d, 64);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), d, 64);
                x |= ((unsigned long long)hi << 32) | lo;
            }
            if (lane_id() == 0) s_q[threadIdx.x / 64] = x;
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int i = 0; i < GFR_WAVES; ++i) x |= s_q[i];
                a.actp[blockIdx.x] = x;
                __threadfence();
            }
            return;
        }
        if (a.ctl->mode != BS_SPLIT) return;
        __shared__ uint32_t s_k[GFR_WAVES], s_m[GFR_WAVES];
        const uint32_t k = wave_sum_u32(kept), mn = wave_min_u32(kmin);
        if (lane_id() == 0) {
            s_k[threadIdx.x / 64] = k;
            s_m[threadIdx.x / 64] = mn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tk = 0, tm = 0xFFFFFFFFu;
            for (int i = 0; i < GFR_WAVES; ++i) {
                tk += s_k[i];
                tm = min(tm, s_m[i]);
            }
            if (tk) {
                atomicAdd(&a.ctl->split_kept, tk);
                atomicMin(&a.ctl->split_min, tm);
            }
            __threadfence();
        }
    }

    __device__ void control(uint32_t nf2, uint32_t mf2) const
    {
        BsCtl *ctl = a.ctl;
        const uint32_t mode = ctl->mode;
        uint32_t imp = 0, far = 0;
        unsigned long long lr = 0;
        if (mode == BS_RELAX) {
            for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) {
                imp += a.part[4 * i];
                far += a.part[4 * i + 1];
                lr += a.part[4 * i + 2];
            }
            __shared__ uint32_t s_i[GFR_WAVES], s_f[GFR_WAVES];
            __shared__ unsigned long long s_l[GFR_WAVES];
            imp = wave_sum_u32(imp);
            far = wave_sum_u32(far);
            lr = wave_sum_u64(lr);
            if (lane_id() == 0) {
                s_i[threadIdx.x / 64] = imp;
                s_f[threadIdx.x / 64] = far;
                s_l[threadIdx.x / 64] = lr;
            }
            __syncthreads();
            imp = far = 0;
            lr = 0;
            for (int i = 0; i < GFR_WAVES; ++i) {
                imp += s_i[i];
                far += s_f[i];
                lr += s_l[i];
            }
        }
        unsigned long long act = 0;
        if (mode == BS_RELAX) {
            for (uint32_t i = threadIdx.x; i < nactp; i += GFR_BLOCK) act |= a.actp[i];
            __shared__ unsigned long long s_a[GFR_WAVES];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)act, d, 64);
                const uint32_t hi2 = (uint32_t)__shfl_xor((int)(uint32_t)(act >> 32), d, 64);
                act |= ((unsigned long long)hi2 << 32) | lo;
            }
            if (lane_id() == 0) s_a[threadIdx.x / 64] = act;
            __syncthreads();
            for (int i = 0; i < GFR_WAVES; ++i) act |= s_a[i];
        }
        if (threadIdx.x != 0) return;
        if (mode == BS_RELAX) ctl->active = act;
        const uint32_t D = ctl->delta, hi = ctl->hi;
        uint32_t split_min = 0xFFFFFFFFu;
        if (mode == BS_RELAX) {
            ctl->relaxed += ctl->dir == BS_PULL ? ctl->m : ctl->mf;
            ctl->pull_iters += ctl->dir == BS_PULL ? 1u : 0u;
            ctl->improvements += imp;
            ctl->lane_relaxed += lr;
            if (far) ctl->far_any = 1u;
        } else {
            ctl->far_any = atomicAdd(&ctl->split_kept, 0u) != 0u;
            split_min = atomicAdd(&ctl->split_min, 0u);
            ctl->split_kept = 0u;
            ctl->split_min = 0xFFFFFFFFu;
            ctl->splits += 1u;
        }
        uint32_t nm;
        if (ctl->overflow) {
            nm = BS_DONE;
        } else if (nf2 > 0) {
            nm = BS_RELAX;
        } else if (ctl->far_any) {
            nm = BS_SPLIT;
            unsigned long long nhi = (unsigned long long)hi + D;
            if (mode == BS_SPLIT && split_min != 0xFFFFFFFFu) {
                const unsigned long long j = ((unsigned long long)split_min / D + 1ull) * D;
                if (j > nhi) nhi = j;
            }
            ctl->lo = hi;
            ctl->hi = nhi > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)nhi;
        } else {
            nm = BS_DONE;
        }
        ctl->nf = nf2;
        ctl->mf = mf2;
        ctl->iter += 1u;
        ctl->parity ^= 1u;
        ctl->mode = nm;
        // a frontier carrying most of the edges is relaxed by a pull sweep
        ctl->dir = (ctl->pull_alpha > 0.f && (double)mf2 * ctl->pull_alpha > (double)ctl->m) ? BS_PULL : BS_PUSH;
    }
};

template <int BITS>
__global__ void bsssp_init(BsArgs a, const int32_t *src, int32_t k, uint32_t delta, float pull_alpha)
{
    if (threadIdx.x == 0) {
        for (int32_t q = 0; q < k; ++q) {
            const int32_t v = src[q];
            bs_store<BITS>(a, (size_t)v, q, 0u);
            a.nq[v] |= 1ull << q;
            a.nany[v] = 1;
        }
        BsCtl *ctl = a.ctl;
        ctl->mode = BS_RELAX;
        ctl->nf = ctl->mf = 0;
        ctl->iter = 0;
        ctl->lo = 0;
        ctl->hi = delta;
        ctl->delta = delta;
        ctl->far_any = 0;
        ctl->split_kept = 0;
        ctl->split_min = 0xFFFFFFFFu;
        ctl->overflow = ctl->parity = ctl->err = ctl->splits = 0;
        ctl->unfit = 0;
        ctl->relaxed = ctl->improvements = ctl->pair_entries = ctl->lane_relaxed = 0ull;
        ctl->active = 0ull;
        ctl->dir = BS_PUSH;
        ctl->pull_alpha = pull_alpha;
        ctl->m = (unsigned long long)a.R[a.n];
        ctl->pull_iters = 0;
    }
}

// out[q][v] = D[v][q] for the queries q in `lanes`: 64 vertices x 64 queries
// per tile through LDS (narrow rows widened, unreached -> 0xFFFFFFFF)
template <int BITS>
__global__ __launch_bounds__(GFR_BLOCK) void bsssp_transpose(BsArgs a, int32_t n, unsigned long long lanes,
                                                             uint32_t *out)
{
    __shared__ uint32_t tile[64][65];
    const int32_t ntiles = (n + 63) / 64;
    for (int32_t tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
        const int32_t v0 = tb * 64;
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 64; i += GFR_BLOCK) {
            const int r = i / 64, q = i % 64;
            tile[r][q] = (v0 + r < n) ? bs_load<BITS>(a, (size_t)(v0 + r), q) : 0u;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 64; i += GFR_BLOCK) {
            const int q = i / 64, r = i % 64;
            if (((lanes >> q) & 1ull) && v0 + r < n) out[(size_t)q * n + v0 + r] = tile[r][q];
        }
    }
}

// A relaxation whose sum does not fit below 0xFFFFFFFF is not applied; the
// batch fails only if such a sum was a shortest distance: for some query in
// `lanes`, a vertex left unreached next to a reached one.  Wave per vertex,
// lane = query.
__global__ __launch_bounds__(GFR_BLOCK) void bsssp_unfit_check(const int32_t *R, const int32_t *C, const uint32_t *D,
                                                                int32_t n, unsigned long long lanes, uint32_t *flag)
{
    const int lane = lane_id();
    const bool mine = (lanes >> lane) & 1ull;
    const uint32_t waves = gridDim.x * GFR_WAVES;
    for (uint32_t v = blockIdx.x * GFR_WAVES + threadIdx.x / 64; v < (uint32_t)n; v += waves) {
        if (!mine || D[(size_t)v * 64 + lane] != BS_INF) continue;
        for (int32_t e = R[v]; e < R[v + 1]; ++e)
            if (D[(size_t)C[e] * 64 + lane] != BS_INF) {
                *flag = 1u;
                break;
            }
    }
}

void run_sssp_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, uint32_t *dist, hipStream_t s)
{
    if (!g.weighted) fail(GFR_E_INVALID, "sssp_batch: graph was loaded without weights");
    const int32_t n = g.n;
    if (k < c.opt.batch_min_sssp) {   // a shared traversal costs about the same for few queries
        for (int32_t i = 0; i < k; ++i) run_sssp(c, g, sources[i], dist + (size_t)i * n, s);
        return;
    }
    const uint32_t chunk = 1024;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    // relax / pull grid per row width: the option's work-groups per CU (or as
    // many as are resident at once), at most one per 1024-edge chunk of the
    // whole graph.  Many more work-groups than fit at once let the hardware
    // hand chunks of uneven cost to whichever CU frees first (R-MAT s22, 64
    // queries: 35.5 ms per batch at 8 per CU, 32.9 at 16, 30.3 at 64).  G
    // sizes the per-work-group partials.
    const int bpc = c.opt.batch_blocks_per_cu;
    const int gcap = (int)std::min<int64_t>(64ll * c.num_cu, std::max<int64_t>(c.num_cu, g.m / 1024 + 1));
    auto grid_of = [&](const void *relax, const void *pull) {
        return std::min(gcap, std::max(resident_grid(c, relax, bpc), resident_grid(c, pull, bpc)));
    };
    const int Gw[3] = {grid_of((const void *)bsssp_relax<1024, 8>, (const void *)bsssp_pull<1024, 8>),
                       grid_of((const void *)bsssp_relax<1024, 16>, (const void *)bsssp_pull<1024, 16>),
                       grid_of((const void *)bsssp_relax<1024, 32>, (const void *)bsssp_pull<1024, 32>)};
    const int G = std::max(Gw[0], std::max(Gw[1], Gw[2]));
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    // one shared bucket serves all queries; a narrow bucket desynchronises the
    // queries' frontiers and multiplies edge visits, so the default is a
    // single bucket (plain frontier order); "batch.delta" sets a width, or
    // "batch.delta_factor" one relative to the mean edge weight
    uint32_t delta = 0xFFFFFFFFu;
    if (c.opt.batch_delta > 0) delta = (uint32_t)c.opt.batch_delta;
    else if (c.opt.batch_delta_factor > 0) delta = sssp_auto_delta(g, c.opt.batch_delta_factor);
    c.arena.reserve(al256(256ull * n) + al256(8ull * n) + 2 * al256(8ull * n) + 2 * al256(32ull * nwords) +
                    3 * al256(4ull * n) + al256(4 * nparts) + al256(16ull * G) + al256(16ull * cg.blocks) +
                    al256(sizeof(BsCtl)) + al256(4 * 64) + al256(8ull * cg.blocks) + al256(4ull * nwords));
    BsArgs a;
    memset(&a, 0, sizeof a);   // padding too: the bytes key the captured steps
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.W = g.W.as<uint32_t>();
    a.n = n;
    a.nwords = nwords;
    a.D = c.arena.take<uint32_t>(64ull * n);
    a.D16 = (uint16_t *)a.D;
    a.D8 = (uint8_t *)a.D;
    a.qm = c.arena.take<unsigned long long>(n);
    a.nq = c.arena.take<unsigned long long>(n);
    a.fq = c.arena.take<unsigned long long>(n);
    a.nany = c.arena.take<uint8_t>(32ull * nwords);
    a.fany = c.arena.take<uint8_t>(32ull * nwords);
    a.q.v = c.arena.take<int32_t>(n);
    a.q.off = c.arena.take<uint32_t>(n);
    a.q.row = c.arena.take<int32_t>(n);
    a.q.part = c.arena.take<int32_t>(nparts);
    a.part = c.arena.take<uint32_t>(4ull * G);
    unsigned long long *status = c.arena.take<unsigned long long>(2ull * cg.blocks);
    a.ctl = c.arena.take<BsCtl>(1);
    int32_t *dsrc = c.arena.take<int32_t>(64);
    a.actp = c.arena.take<unsigned long long>(cg.blocks);
    a.fbits = c.arena.take<uint32_t>(nwords);
    a.pending = c.opt.batch_pending != 0;
    a.sparse = (uint32_t)c.opt.batch_sparse;
    a.full = g.full;
    a.full_nf = (uint32_t)g.full_nf;
    a.full_mf = (uint32_t)g.m;
    double iters = 0, relaxed = 0, imps = 0, pulls = 0, lanes = 0, pairs = 0, fallbacks = 0;
    double batches8 = 0, batches16 = 0;
    // narrow rows first (option batch.narrow: 0 never, 1 auto, 2 always
    // tried first from 16 bits, 3 always tried first from 8 bits); auto skips
    // them on mesh-class graphs, whose long paths outgrow them, and starts a
    // graph at the narrowest width no batch on it has outgrown
    const int nopt = c.opt.batch_narrow;
    int bits = 32;
    if (nopt == 3) bits = 8;
    else if (nopt == 2) bits = 16;
    else if (nopt == 1 && g.cls == GRAPH_SCALEFREE) bits = std::max(8, g.row_bits_min.load());
    const float pull_alpha = (float)c.opt.batch_pull_alpha;
    const bool pair = c.opt.batch_pair != 0;   // 32-bit rows: two edges per row instruction
    for (int32_t g0 = 0; g0 < k; g0 += 64) {
        const int32_t kk = std::min<int32_t>(64, k - g0);
        const unsigned long long lanes_mask = kk == 64 ? ~0ull : ((1ull << kk) - 1ull);
        BsCtl h;
        for (;;) {
            fill_u32(a.D, 0xFFFFFFFFu, 2ull * bits * n, s);   // 8 * bits bytes per vertex
            fill_u32(a.nq, 0u, 2ull * n, s);
            fill_u32(a.fq, 0u, 2ull * n, s);
            fill_u32(a.nany, 0u, 8ull * nwords, s);
            fill_u32(a.fany, 0u, 8ull * nwords, s);
            fill_u32(a.part, 0u, 4ull * G, s);
            fill_u32(status, 0u, 4ull * cg.blocks, s);
            GFR_HIP(hipMemcpyAsync(dsrc, sources + g0, 4ull * kk, hipMemcpyHostToDevice, s));
            auto by_width = [&](auto f) {
                if (bits == 8) f(std::integral_constant<int, 8>());
                else if (bits == 16) f(std::integral_constant<int, 16>());
                else f(std::integral_constant<int, 32>());
            };
            by_width([&](auto B) {
                hipLaunchKernelGGL(bsssp_init<decltype(B)::value>, dim3(1), dim3(64), 0, s, a, dsrc, kk, delta,
                                   pull_alpha);
            });
            auto compact = [&]() {
                c.ktimer.run("bsssp_compact", s, [&]() {
                    by_width([&](auto B) {
                        constexpr int W = decltype(B)::value;
                        hipLaunchKernelGGL(compact_kernel<BsMarks<W>>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, a.R,
                                           n, nwords, cg.wpt, BsMarks<W>{a, (uint32_t)G, cg.blocks, cg.wpt == 1u}, a.q, chunk,
                                           status, &a.ctl->parity, &a.ctl->err);
                    });
                });
            };
            compact();   // queue of the sources
            GFR_LAUNCH_CHECK();
            auto launch = [&]() {
                const int Gb = Gw[bits == 8 ? 0 : bits == 16 ? 1 : 2];
                c.ktimer.run("bsssp_relax", s, [&]() {
                    if (bits == 32 && pair)
                        hipLaunchKernelGGL(bsssp_relax2<1024>, dim3(Gb), dim3(GFR_BLOCK), 0, s, a);
                    else
                        by_width([&](auto B) {
                            hipLaunchKernelGGL((bsssp_relax<1024, decltype(B)::value>), dim3(Gb), dim3(GFR_BLOCK), 0,
                                               s, a);
                        });
                });
                // the pull sweep runs only where the control chose it; with
                // pull_alpha 0 it never does, and is not launched at all
                if (pull_alpha > 0.f)
                    c.ktimer.run("bsssp_pull", s, [&]() {
                        by_width([&](auto B) {
                            hipLaunchKernelGGL((bsssp_pull<1024, decltype(B)::value>), dim3(Gb), dim3(GFR_BLOCK), 0,
                                               s, a);
                        });
                    });
                compact();
            };
            StepKey key("bsssp");
            key.add(a).add(G).add(Gw).add(cg).add(chunk).add(status).add(bits).add(pair).add(pull_alpha);
            run_until_done(c, &a.ctl->mode, BS_DONE, g.bsssp_iter_hint.load(std::memory_order_relaxed) + 1,
                           64ll * n + 1024, s, launch, &key);
            if (bits == 32) {
                // no fallback can follow: the output is written before the
                // control block is read back (a failed batch fails the call)
                hipLaunchKernelGGL(bsssp_transpose<32>, dim3(G), dim3(GFR_BLOCK), 0, s, a, n, lanes_mask,
                                   dist + (size_t)g0 * n);
                GFR_LAUNCH_CHECK();
            }
            GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(BsCtl), hipMemcpyDeviceToHost, s));
            GFR_HIP(hipStreamSynchronize(s));
            memcpy(&h, c.pinned, sizeof(BsCtl));
            if (h.err) fail(GFR_E_DEVICE, "sssp_batch: frontier compaction look-back timed out");
            g.bsssp_iter_hint.store((int32_t)h.iter, std::memory_order_relaxed);
            if (bits < 32 && h.overflow) {
                // a distance outgrew the narrow rows: this batch again, twice as wide
                bits *= 2;
                int cur = g.row_bits_min.load();
                while (cur < bits && !g.row_bits_min.compare_exchange_weak(cur, bits)) {
                }
                fallbacks += 1;
                continue;
            }
            break;
        }
        if (h.unfit) {
            // 32-bit rows (narrow batches fall back instead): was an unfit sum a distance?
            fill_u32(a.part, 0u, 1, s);
            hipLaunchKernelGGL(bsssp_unfit_check, dim3(G), dim3(GFR_BLOCK), 0, s, a.R, a.C, a.D, n, lanes_mask,
                               a.part);
            GFR_LAUNCH_CHECK();
            GFR_HIP(hipMemcpyAsync(c.pinned, a.part, 4, hipMemcpyDeviceToHost, s));
            GFR_HIP(hipStreamSynchronize(s));
            if (*(volatile uint32_t *)c.pinned)
                fail(GFR_E_INVALID, "sssp_batch: a distance does not fit below 0xFFFFFFFF");
        }
        if (bits == 8)
            hipLaunchKernelGGL(bsssp_transpose<8>, dim3(G), dim3(GFR_BLOCK), 0, s, a, n, lanes_mask,
                               dist + (size_t)g0 * n);
        else if (bits == 16)
            hipLaunchKernelGGL(bsssp_transpose<16>, dim3(G), dim3(GFR_BLOCK), 0, s, a, n, lanes_mask,
                               dist + (size_t)g0 * n);
        GFR_LAUNCH_CHECK();
        batches8 += bits == 8 ? 1 : 0;
        batches16 += bits == 16 ? 1 : 0;
        iters += h.iter;
        relaxed += (double)h.relaxed;
        imps += (double)h.improvements;
        pulls += h.pull_iters;
        lanes += (double)h.lane_relaxed;
        pairs += (double)h.pair_entries;
    }
    c.stats.v["narrow_batches"] += batches8 + batches16;   // batches finished with 8- or 16-bit rows
    c.stats.v["batches_8bit"] += batches8;
    c.stats.v["batches_16bit"] += batches16;
    c.stats.v["narrow_fallbacks"] += fallbacks;            // batches solved again with wider rows
    c.stats.v["iterations"] += iters;
    c.stats.v["relaxations"] += relaxed;   // edge visits, each serving up to 64 queries
    c.stats.v["lane_relaxations"] += lanes;   // (edge, query) relaxations
    c.stats.v["pair_entries"] += pairs;       // (vertex, query) entries of the near queues
    c.stats.v["improvements"] += imps;
    c.stats.v["pull_iterations"] += pulls;
    c.stats.v["solves"] += k;
}

// ---------------------------------------------------------------- sessions
// Lanes of a session join between relaxation rounds: their distance column is
// reset, the source gets distance 0 and a mark, and the next compaction puts
// it into the near queue.  A session uses one bucket (frontier order), so a
// lane with no queued (vertex, lane) pair is finished and its column final.

__global__ __launch_bounds__(GFR_BLOCK) void bs_clear_lanes(uint32_t *D, int32_t n, unsigned long long lanes)
{
    const int lane = lane_id();
    const bool mine = (lanes >> lane) & 1ull;
    const uint32_t waves = gridDim.x * GFR_WAVES;
    for (uint32_t v = blockIdx.x * GFR_WAVES + threadIdx.x / 64; v < (uint32_t)n; v += waves)
        if (mine) D[(size_t)v * 64 + lane] = 0xFFFFFFFFu;
}

__global__ void bs_admit(BsArgs a, const int32_t *pairs, int32_t count)
{
    if (threadIdx.x != 0) return;
    for (int32_t i = 0; i < count; ++i) {
        const int32_t q = pairs[2 * i], src = pairs[2 * i + 1];
        a.D[(size_t)src * 64 + q] = 0u;
        a.nq[src] |= 1ull << q;
        a.nany[src] = 1;
    }
    BsCtl *ctl = a.ctl;
    if (count && ctl->mode == BS_DONE) {
        ctl->mode = BS_RELAX;
        ctl->nf = ctl->mf = 0;
    }
}

__global__ void bs_session_init(BsArgs a, float pull_alpha)
{
    if (threadIdx.x != 0) return;
    BsCtl *ctl = a.ctl;
    ctl->mode = BS_DONE;
    ctl->nf = ctl->mf = 0;
    ctl->iter = 0;
    ctl->lo = 0;
    ctl->hi = ctl->delta = 0xFFFFFFFFu;
    ctl->far_any = 0;
    ctl->split_kept = 0;
    ctl->split_min = 0xFFFFFFFFu;
    ctl->overflow = ctl->parity = ctl->err = ctl->splits = 0;
    ctl->unfit = 0;
    ctl->relaxed = ctl->improvements = ctl->pair_entries = ctl->lane_relaxed = 0ull;
    ctl->active = 0ull;
    ctl->dir = BS_PUSH;
    ctl->pull_alpha = pull_alpha;
    ctl->m = (unsigned long long)a.R[a.n];
    ctl->pull_iters = 0;
}

namespace {
struct BsLayout {
    size_t n, nwords, nparts, G, blocks;
    size_t total() const
    {
        return al256(256 * n) + al256(8 * n) + 2 * al256(8 * n) + 2 * al256(32 * nwords) + 3 * al256(4 * n) +
               al256(4 * nparts) + al256(16 * G) + al256(16 * blocks) + al256(sizeof(BsCtl)) + al256(8 * blocks) +
               al256(4 * 128) + al256(4 * 64 * n) + al256(4 * nwords);
    }
};
BsLayout bs_layout(int64_t n, int64_t m, int num_cu)
{
    BsLayout L;
    L.n = (size_t)n;
    L.nwords = (size_t)((n + 63) / 64) * 2;
    L.nparts = (size_t)(m / 1024) + 2;
    // relax grid as for direct batches: 64 work-groups per CU, at most one per 1024-edge chunk
    L.G = (size_t)std::min<int64_t>(64ll * num_cu, std::max<int64_t>(num_cu, m / 1024 + 1));
    L.blocks = compact_geom((uint32_t)L.nwords, num_cu).blocks;
    return L;
}
}  // namespace

uint64_t sssp_session_bytes(int64_t n, int64_t m, int num_cu) { return bs_layout(n, m, num_cu).total(); }

struct BsSession final : LaneSession {
    Ctx &c;
    Graph &g;
    DevMem mem;
    BsArgs a{};
    CompactGeom cg{};
    int G = 0;
    bool pull = false;   // pull sweeps possible (batch.pull_alpha > 0)
    uint32_t nwords = 0;
    unsigned long long *status = nullptr;
    int32_t *pairs = nullptr, *pin_pairs = nullptr;
    BsCtl *pin = nullptr;

    BsSession(Ctx &cc, Graph &gg, const Options &o) : c(cc), g(gg)
    {
        if (!g.weighted) fail(GFR_E_INVALID, "sssp query: graph was loaded without weights");
        n = g.n;
        const BsLayout L = bs_layout(g.n, g.m, c.num_cu);
        nwords = (uint32_t)L.nwords;
        G = (int)L.G;
        cg = compact_geom(nwords, c.num_cu);
        bytes = L.total();
        GFR_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        GFR_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        GFR_HIP(hipHostMalloc((void **)&pin, sizeof(BsCtl), hipHostMallocDefault));
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
        a.W = g.W.as<uint32_t>();
        a.n = g.n;
        a.nwords = nwords;
        a.D = (uint32_t *)take(256 * L.n);
        a.D16 = nullptr;   // sessions keep 32-bit rows (lanes join at different times; no batch to solve again)
        a.D8 = nullptr;
        a.qm = (unsigned long long *)take(8 * L.n);
        a.nq = (unsigned long long *)take(8 * L.n);
        a.fq = (unsigned long long *)take(8 * L.n);
        a.nany = (uint8_t *)take(32 * L.nwords);
        a.fany = (uint8_t *)take(32 * L.nwords);
        a.q.v = (int32_t *)take(4 * L.n);
        a.q.off = (uint32_t *)take(4 * L.n);
        a.q.row = (int32_t *)take(4 * L.n);
        a.q.part = (int32_t *)take(4 * L.nparts);
        a.part = (uint32_t *)take(16 * L.G);
        status = (unsigned long long *)take(16 * L.blocks);
        a.ctl = (BsCtl *)take(sizeof(BsCtl));
        a.actp = (unsigned long long *)take(8 * L.blocks);
        pairs = (int32_t *)take(4 * 128);
        stage = take(4 * 64 * L.n);
        a.fbits = (uint32_t *)take(4 * L.nwords);
        a.pending = o.batch_pending != 0;
        a.sparse = (uint32_t)o.batch_sparse;
        a.full = g.full;
        a.full_nf = (uint32_t)g.full_nf;
        a.full_mf = (uint32_t)g.m;
        fill_u32(a.D, 0xFFFFFFFFu, 64 * L.n, stream);
        fill_u32(a.nq, 0u, 2 * L.n, stream);
        fill_u32(a.fq, 0u, 2 * L.n, stream);
        fill_u32(a.nany, 0u, 8 * L.nwords, stream);
        fill_u32(a.fany, 0u, 8 * L.nwords, stream);
        fill_u32(a.part, 0u, 4 * L.G, stream);
        fill_u32(status, 0u, 4 * L.blocks, stream);
        pull = o.batch_pull_alpha > 0;
        hipLaunchKernelGGL(bs_session_init, dim3(1), dim3(64), 0, stream, a, (float)o.batch_pull_alpha);
        GFR_LAUNCH_CHECK();
    }
    ~BsSession() override
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
        GFR_HIP(hipStreamSynchronize(stream));   // the pinned staging of the last admission is consumed
        unsigned long long mask = 0;
        for (int32_t i = 0; i < count; ++i) {
            pin_pairs[2 * i] = lanes[i];
            pin_pairs[2 * i + 1] = sources[i];
            mask |= 1ull << lanes[i];
        }
        GFR_HIP(hipMemcpyAsync(pairs, pin_pairs, 8ull * count, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(bs_clear_lanes, dim3(G), dim3(GFR_BLOCK), 0, stream, a.D, a.n, mask);
        hipLaunchKernelGGL(bs_admit, dim3(1), dim3(64), 0, stream, a, pairs, count);
        GFR_LAUNCH_CHECK();
    }
    void release(unsigned long long) override {}   // a finished lane has no queued pairs left
    void enqueue_step() override
    {
        hipLaunchKernelGGL((bsssp_relax<1024, 32>), dim3(G), dim3(GFR_BLOCK), 0, stream, a);
        if (pull) hipLaunchKernelGGL((bsssp_pull<1024, 32>), dim3(G), dim3(GFR_BLOCK), 0, stream, a);
        hipLaunchKernelGGL(compact_kernel<BsMarks<32>>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, stream, a.R, a.n,
                           nwords, cg.wpt, BsMarks<32>{a, (uint32_t)G, cg.blocks, cg.wpt == 1u}, a.q, 1024u, status,
                           &a.ctl->parity, &a.ctl->err);
        GFR_LAUNCH_CHECK();
        GFR_HIP(hipMemcpyAsync(pin, a.ctl, sizeof(BsCtl), hipMemcpyDeviceToHost, stream));
    }
    unsigned long long active() const override { return pin->mode == BS_DONE ? 0ull : pin->active; }
    gfr_status failed(std::string &msg) const override
    {
        if (pin->err) {
            msg = "sssp query: frontier compaction look-back timed out";
            return GFR_E_DEVICE;
        }
        if (pin->overflow || pin->unfit) {
            // a session has no per-lane check: a sum past 32 bits fails its queries
            msg = "sssp query: a path weight does not fit below 0xFFFFFFFF";
            return GFR_E_INVALID;
        }
        return GFR_OK;
    }
    void extract(unsigned long long lanes) override
    {
        if (!lanes) return;
        hipLaunchKernelGGL(bsssp_transpose<32>, dim3(G), dim3(GFR_BLOCK), 0, stream, a, a.n, lanes,
                           (uint32_t *)stage);
        GFR_LAUNCH_CHECK();
    }
};

std::unique_ptr<LaneSession> make_sssp_session(Ctx &c, Graph &g, const Options &o)
{
    return std::unique_ptr<LaneSession>(new BsSession(c, g, o));
}

}  // namespace gfr
