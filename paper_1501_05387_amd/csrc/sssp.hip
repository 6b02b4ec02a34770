// sssp.hip -- single-source shortest paths with a near/far priority queue
// (Sec. 4.1 Algorithm 1 for the advance/filter/priority-queue sequence,
// Sec. 4.5 "Priority Queue" for the near/far split, Sec. 5.2).
//
// Every iteration is two launches:
//   sssp_relax   the advance over the near queue with the same load-balanced
//                edge chunks as BFS; each edge does
//                atomicMin(dist[v], dist[u] + w) and, if that improved v, marks
//                v (one plain byte store) as near when its new distance is
//                inside the current bucket, otherwise as far.  Marks stand in
//                for the flag array of Sec. 5.2 that removes redundant
//                vertices: many improvers of one vertex leave one mark.
//   compact      the filter.  In a relax iteration it consumes the near marks
//                into the next near queue (vertex order).  When the near queue
//                has run dry the bucket advances by delta and the same kernel
//                splits the far marks instead: settled entries are dropped,
//                entries inside the new bucket become the near queue, the rest
//                stay far (Sec. 4.5).  The last work-group runs the control.
// The host enqueues iterations speculatively (see bfs.hip).
#include "compact.h"
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { SS_RELAX = 0, SS_SPLIT = 1, SS_DONE = 2 };

struct SsspCtl {
    uint32_t mode;               // SS_* (first word: read back by the host)
    uint32_t nf, mf;             // entries / edges of the current near queue
    uint32_t iter;
    uint32_t lo, hi;             // current bucket [lo, hi)
    uint32_t delta;
    uint32_t far_any;            // the far set may be non-empty
    uint32_t split_kept;         // far vertices left by the running split
    uint32_t split_seen;         // far vertices examined by the running split
    uint32_t split_min;          // smallest distance among them
    uint32_t unfit;              // a relaxation's sum did not fit below 0xFFFFFFFF (checked after the solve)
    uint32_t parity;
    uint32_t err;
    uint32_t splits;
    // traffic model counters
    unsigned long long near_entries, relaxed, improvements, far_entries;
    uint32_t dir;                // SS_PUSH / SS_PULL for the next relaxation
    float pull_alpha;            // pull when the near queue's edges exceed m / pull_alpha (0: never)
    unsigned long long m;
    uint32_t pull_iters, pad;
};

enum : uint32_t { SS_PUSH = 0, SS_PULL = 1 };

struct SsspArgs {
    const int32_t *R;
    const int32_t *C;
    const uint32_t *W;
    int32_t n;
    uint32_t nwords;
    uint32_t *dist;
    uint8_t *near;         // marks of the near queue being built, one byte per vertex
    uint8_t *far;          // marks of the far set
    FrontierQ q;
    uint32_t *part;        // per work-group [improvements, far marks written]
    SsspCtl *ctl;
    uint32_t *fbits;       // [nwords] bitmap of the near queue (written by the compaction)
    FrontierQ full;        // every vertex with edges (pull sweeps)
    uint32_t full_nf, full_mf;
};

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void sssp_relax(SsspArgs a)
{
    SsspCtl *ctl = a.ctl;
    if (ctl->mode != SS_RELAX || ctl->dir != SS_PUSH) return;
    const uint32_t hi = ctl->hi, nf = ctl->nf, mf = ctl->mf;
    const FrontierQ q = a.q;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ uint32_t s_du[CH + 1];
    const uint32_t nchunks = (mf + CH - 1) / CH;
    bool ovf = false;
    uint32_t nimp = 0, nfar = 0;
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
            s_du[i] = a.dist[q.v[s + i]];
        }
        __syncthreads();
        // each thread takes every GFR_BLOCK-th edge of the chunk: all its
        // column and weight loads are issued first, then all distance probes,
        // and the tests are computed for every edge so that no load is moved
        // into a branch and waited for there (an edge past the chunk end
        // repeats the chunk's first edge and is masked)
        constexpr int PER = CH / GFR_BLOCK;
        int32_t vv[PER];
        uint32_t nd[PER], dv[PER];
        bool ok[PER], fits[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const uint32_t e = e0 + p * GFR_BLOCK + threadIdx.x;
            ok[p] = e < e1;
            const uint32_t ec = ok[p] ? e : e0;
            const int i = upper_index(s_off, 0, cnt - 1, ec);
            const int32_t idx = s_row[i] + (int32_t)(ec - s_off[i]);
            vv[p] = a.C[idx];
            const unsigned long long nd64 = (unsigned long long)s_du[i] + a.W[idx];
            fits[p] = nd64 < 0xFFFFFFFFull;
            nd[p] = (uint32_t)nd64;
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) dv[p] = a.dist[vv[p]];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            ovf |= ok[p] & !fits[p];
            // non-returning atomicMin; marking on the pre-check marks a
            // superset of the true improvements, which only re-relaxes such
            // a vertex with its current distance
            if (ok[p] & fits[p] & (nd[p] < dv[p])) {
                atomicMin(a.dist + vv[p], nd[p]);
                ++nimp;
                if (nd[p] < hi) {
                    a.near[vv[p]] = 1;
                } else {
                    a.far[vv[p]] = 1;
                    ++nfar;
                }
            }
        }
    }
    if (ovf) ctl->unfit = 1u;
    __shared__ uint32_t s_a[GFR_WAVES], s_b[GFR_WAVES];
    nimp = wave_sum_u32(nimp);
    nfar = wave_sum_u32(nfar);
    if (lane_id() == 0) {
        s_a[threadIdx.x / 64] = nimp;
        s_b[threadIdx.x / 64] = nfar;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0, y = 0;
        for (int i = 0; i < GFR_WAVES; ++i) {
            x += s_a[i];
            y += s_b[i];
        }
        a.part[2 * blockIdx.x] = x;
        a.part[2 * blockIdx.x + 1] = y;
    }
}

// Pull relaxation (Sec. 4.5's pull advance applied to SSSP, which the paper
// leaves to future work): for near queues that carry most of the edges, a
// load-balanced sweep over every vertex's list.  An edge (v, u) whose u is
// in the near queue (bitmap) offers dist[u] + w to v; each wave forms the
// minimum offer per owner v over its 64 edges with a segmented scan, and the
// last lane of each owner's run lowers dist[v] once (pre-checked atomicMin)
// and marks it near or far.  Sources outside the queue cost one bitmap probe.
template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void sssp_pull(SsspArgs a)
{
    SsspCtl *ctl = a.ctl;
    if (ctl->mode != SS_RELAX || ctl->dir != SS_PULL) return;
    const uint32_t hi = ctl->hi;
    const FrontierQ q = a.full;
    const uint32_t nf = a.full_nf, mf = a.full_mf;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    constexpr uint32_t QW = CH / GFR_WAVES;
    const uint32_t nchunks = (mf + CH - 1) / CH;
    bool unf = false;
    uint32_t nimp = 0, nfar = 0;
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
            const int nb = (int)min(64u, ee - e);
            int32_t v = -1;
            uint32_t offer = 0xFFFFFFFFu;
            int il = ilo;
            if (lane < nb) {
                const uint32_t el = e + lane;
                il = upper_index(s_off, ilo, min(cnt - 1, ilo + lane + 1), el);
                const int32_t idx = s_row[il] + (int32_t)(el - s_off[il]);
                const int32_t u = a.C[idx];
                v = s_v[il];
                if ((a.fbits[u >> 5] >> (u & 31)) & 1u) {
                    const unsigned long long s64 = (unsigned long long)a.dist[u] + a.W[idx];
                    if (s64 < 0xFFFFFFFFull) offer = (uint32_t)s64;
                    else unf = true;
                }
            }
            ilo = __builtin_amdgcn_readlane(il, nb - 1);
            // segmented minimum over runs of equal owners (lanes are in edge order)
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = (uint32_t)__shfl_up((int)offer, d, 64);
                const int32_t ov = __shfl_up(v, d, 64);
                if (lane >= d && ov == v) offer = min(offer, o);
            }
            const int32_t vnext = __shfl_down(v, 1, 64);
            const bool last = lane < nb && (lane == nb - 1 || vnext != v);
            if (last && offer != 0xFFFFFFFFu && offer < a.dist[v]) {
                atomicMin(a.dist + v, offer);
                ++nimp;
                if (offer < hi) {
                    a.near[v] = 1;
                } else {
                    a.far[v] = 1;
                    ++nfar;
                }
            }
        }
    }
    if (unf) ctl->unfit = 1u;
    __shared__ uint32_t s_a[GFR_WAVES], s_b[GFR_WAVES];
    nimp = wave_sum_u32(nimp);
    nfar = wave_sum_u32(nfar);
    if (lane == 0) {
        s_a[wave] = nimp;
        s_b[wave] = nfar;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0, y = 0;
        for (int i = 0; i < GFR_WAVES; ++i) {
            x += s_a[i];
            y += s_b[i];
        }
        a.part[2 * blockIdx.x] = x;
        a.part[2 * blockIdx.x + 1] = y;
    }
}

struct SsspMarks {
    SsspArgs a;
    uint32_t nparts;   // work-groups of sssp_relax
    // per-thread split results
    uint32_t kept = 0;
    uint32_t seen = 0;
    uint32_t kmin = 0xFFFFFFFFu;

    __device__ bool skip() const { return a.ctl->mode == SS_DONE; }

    __device__ uint32_t mask(uint32_t w)
    {
        SsspCtl *ctl = a.ctl;
        if (ctl->mode == SS_RELAX) {   // consume the near marks
            const uint32_t m = marks_to_mask(a.near + 32ull * w);
            a.fbits[w] = m;
            if (m) clear_marks(a.near + 32ull * w);
            return m;
        }
        // split the far marks with the new bucket [lo, hi)
        const uint32_t f = marks_to_mask(a.far + 32ull * w);
        if (!f) {
            a.fbits[w] = 0u;
            return 0u;
        }
        const uint32_t lo = ctl->lo, hi = ctl->hi;
        uint32_t out = 0, bits = f;
        seen += __popc(f);
        while (bits) {
            const int bi = __ffs(bits) - 1;
            bits &= bits - 1;
            const uint32_t v = w * 32u + bi;
            const uint32_t d = a.dist[v];
            if (d < hi) {
                a.far[v] = 0;
                if (d >= lo) out |= 1u << bi;
            } else {
                ++kept;
                kmin = min(kmin, d);
            }
        }
        a.fbits[w] = out;
        return out;
    }

    __device__ void partial(uint32_t)
    {
        if (a.ctl->mode != SS_SPLIT) return;
        __shared__ uint32_t s_k[GFR_WAVES], s_m[GFR_WAVES], s_s[GFR_WAVES];
        const uint32_t k = wave_sum_u32(kept), mn = wave_min_u32(kmin), sn = wave_sum_u32(seen);
        if (lane_id() == 0) {
            s_k[threadIdx.x / 64] = k;
            s_m[threadIdx.x / 64] = mn;
            s_s[threadIdx.x / 64] = sn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tk = 0, tm = 0xFFFFFFFFu, ts = 0;
            for (int i = 0; i < GFR_WAVES; ++i) {
                tk += s_k[i];
                tm = min(tm, s_m[i]);
                ts += s_s[i];
            }
            if (tk) {
                atomicAdd(&a.ctl->split_kept, tk);
                atomicMin(&a.ctl->split_min, tm);
            }
            if (ts) atomicAdd(&a.ctl->split_seen, ts);
            __threadfence();   // the split totals are visible before this group publishes
        }
    }

    __device__ void control(uint32_t nf2, uint32_t mf2) const
    {
        SsspCtl *ctl = a.ctl;
        const uint32_t mode = ctl->mode;
        uint32_t imp = 0, far = 0;
        if (mode == SS_RELAX) {
            for (uint32_t i = threadIdx.x; i < nparts; i += GFR_BLOCK) {
                imp += a.part[2 * i];
                far += a.part[2 * i + 1];
            }
            __shared__ uint32_t s_i[GFR_WAVES], s_f[GFR_WAVES];
            imp = wave_sum_u32(imp);
            far = wave_sum_u32(far);
            if (lane_id() == 0) {
                s_i[threadIdx.x / 64] = imp;
                s_f[threadIdx.x / 64] = far;
            }
            __syncthreads();
            imp = far = 0;
            for (int i = 0; i < GFR_WAVES; ++i) {
                imp += s_i[i];
                far += s_f[i];
            }
        }
        if (threadIdx.x != 0) return;
        const uint32_t D = ctl->delta, hi = ctl->hi;
        uint32_t split_min = 0xFFFFFFFFu;
        if (mode == SS_RELAX) {
            ctl->near_entries += ctl->nf;
            ctl->relaxed += ctl->dir == SS_PULL ? ctl->m : ctl->mf;
            ctl->pull_iters += ctl->dir == SS_PULL ? 1u : 0u;
            ctl->improvements += imp;
            if (far) ctl->far_any = 1u;
        } else {
            ctl->far_entries += atomicAdd(&ctl->split_seen, 0u);
            ctl->far_any = atomicAdd(&ctl->split_kept, 0u) != 0u;
            split_min = atomicAdd(&ctl->split_min, 0u);
            ctl->split_kept = 0u;
            ctl->split_seen = 0u;
            ctl->split_min = 0xFFFFFFFFu;
            ctl->splits += 1u;
        }
        uint32_t nm;
        if (nf2 > 0) {
            nm = SS_RELAX;
        } else if (ctl->far_any) {
            nm = SS_SPLIT;
            unsigned long long nhi = (unsigned long long)hi + D;
            if (mode == SS_SPLIT && split_min != 0xFFFFFFFFu) {
                // nothing fell into the bucket: jump to the one holding the smallest far distance
                const unsigned long long j = ((unsigned long long)split_min / D + 1ull) * D;
                if (j > nhi) nhi = j;
            }
            ctl->lo = hi;
            ctl->hi = nhi > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)nhi;
        } else {
            nm = SS_DONE;
        }
        ctl->nf = nf2;
        ctl->mf = mf2;
        ctl->iter += 1u;
        ctl->parity ^= 1u;
        ctl->mode = nm;
        // a near queue carrying most of the edges is relaxed by a pull sweep
        ctl->dir = (ctl->pull_alpha > 0.f && (double)mf2 * ctl->pull_alpha > (double)ctl->m) ? SS_PULL : SS_PUSH;
    }
};

__global__ void sssp_init(SsspArgs a, int32_t src, uint32_t chunk, uint32_t delta, float pull_alpha)
{
    const int32_t rs = a.R[src], deg = a.R[src + 1] - rs;
    if (threadIdx.x == 0) {
        SsspCtl *ctl = a.ctl;
        a.dist[src] = 0u;
        a.q.v[0] = src;
        a.q.off[0] = 0;
        a.q.row[0] = rs;
        ctl->nf = 1;
        ctl->mf = (uint32_t)deg;
        ctl->iter = 0;
        ctl->lo = 0;
        ctl->hi = delta;
        ctl->delta = delta;
        ctl->far_any = 0;
        ctl->split_kept = 0;
        ctl->split_seen = 0;
        ctl->split_min = 0xFFFFFFFFu;
        ctl->unfit = 0;
        ctl->parity = 0;
        ctl->err = 0;
        ctl->splits = 0;
        ctl->near_entries = ctl->relaxed = ctl->improvements = ctl->far_entries = 0ull;
        ctl->dir = SS_PUSH;
        ctl->pull_alpha = pull_alpha;
        ctl->m = (unsigned long long)a.R[a.n];
        ctl->pull_iters = 0;
        ctl->mode = deg == 0 ? SS_DONE : SS_RELAX;
    }
    // (the first iteration pushes; every compaction writes the near-queue bitmap a pull reads)
    for (uint32_t c = threadIdx.x; (uint64_t)c * chunk < (uint64_t)deg; c += blockDim.x) a.q.part[c] = 0;
}

uint32_t sssp_auto_delta(const Graph &g, double factor)
{
    double d = g.mean_w * factor;
    if (d < 1.0) d = 1.0;
    if (d > 1.0e9) d = 1.0e9;
    return (uint32_t)d;
}

// A relaxation whose sum does not fit below 0xFFFFFFFF is not applied.  The
// solve fails only if that sum was some vertex's shortest distance: a
// vertex left unreached next to a reached one (every sum into it overflowed).
__global__ __launch_bounds__(GFR_BLOCK) void sssp_unfit_check(const int32_t *R, const int32_t *C,
                                                               const uint32_t *dist, int32_t n, uint32_t *flag)
{
    const int32_t stride = (int32_t)(gridDim.x * blockDim.x);
    for (int32_t v = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); v < n; v += stride) {
        if (dist[v] != 0xFFFFFFFFu) continue;
        for (int32_t e = R[v]; e < R[v + 1]; ++e)
            if (dist[C[e]] != 0xFFFFFFFFu) {
                *flag = 1u;
                break;
            }
    }
}

// flag: one device word of the solve's scratch
static void sssp_check_unfit(Ctx &c, Graph &g, const uint32_t *dist, uint32_t *flag, hipStream_t s)
{
    fill_u32(flag, 0u, 1, s);
    hipLaunchKernelGGL(sssp_unfit_check, dim3(grid_blocks(c, 4)), dim3(GFR_BLOCK), 0, s, g.R.as<int32_t>(),
                       g.C.as<int32_t>(), dist, g.n, flag);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, flag, 4, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    if (*(volatile uint32_t *)c.pinned) fail(GFR_E_INVALID, "sssp: a distance does not fit below 0xFFFFFFFF");
}

// ------------------------------------------------------------ mark-byte levels
// Option sssp.frontier 2: the frontier stays as mark bytes and an iteration
// is one launch, as for the mark-byte BFS levels: a launch
// scans the current near marks (consuming them), lists the marked vertices
// in LDS and relaxes each one's edges, marking improved vertices near
// (distance inside the bucket) or far.  A launch that follows one which
// marked nothing near splits instead (Sec. 4.5): the bucket moves past the
// smallest far distance, far-marked vertices inside it are relaxed, those
// beyond it keep their marks, those below it (relaxed since) drop theirs.
// No launch waits for another work-group: every work-group of launch L reads
// the per-group words of launch L-1 and derives the same mode and bucket.

enum : uint32_t { SM_RELAX = 0, SM_SPLIT = 1, SM_DONE = 2 };

struct SmState {
    uint32_t mode, hi;            // this launch's mode and bucket bound [.., hi)
    uint32_t far_any, far_min;    // far marks (may) remain from before this launch; their smallest distance
};

struct SmCtl {
    uint32_t done;                // read back by the host
    uint32_t unfit;               // a relaxation's sum did not fit below 0xFFFFFFFF (checked after the solve)
    uint32_t iter, splits;
    unsigned long long near_entries, relaxed, improvements, far_entries;
};

struct SmArgs {
    const int32_t *R;
    const int32_t *C;
    const uint32_t *W;
    int32_t n;
    uint32_t *dist;
    uint8_t *mk[2];               // near marks by launch parity (n rounded up to 16 bytes)
    uint8_t *far;                 // far marks
    unsigned long long *flags;    // [2][G]: (smallest far distance marked or kept) << 32 | bits, by parity
    SmState *st;                  // [2] by parity, written by work-group 0
    SmCtl *ctl;
    uint32_t delta;
};

enum : uint32_t { SMF_NEAR = 1, SMF_FAR = 2 };

__global__ void sssp_marks_init(SmArgs a, int32_t src, uint32_t G)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    // the launch "before" launch 0 marked the source near in work-group 0
    if (i < G) a.flags[G + i] = i == 0 ? (0xFFFFFFFFull << 32) | SMF_NEAR : (0xFFFFFFFFull << 32);
    if (i == 0) {
        a.dist[src] = 0u;
        a.mk[0][src] = 1;
        a.st[1] = SmState{SM_RELAX, a.delta, 0u, 0xFFFFFFFFu};
        SmCtl *ctl = a.ctl;
        ctl->done = 0;
        ctl->unfit = 0;
        ctl->iter = ctl->splits = 0;
        ctl->near_entries = ctl->relaxed = ctl->improvements = ctl->far_entries = 0ull;
    }
}

__global__ __launch_bounds__(GFR_BLOCK) void sssp_mark_level(SmArgs a, int32_t L)
{
    const uint32_t G = gridDim.x;
    const int lane = lane_id(), wave = threadIdx.x / 64;
    __shared__ uint32_t s_bits[GFR_WAVES], s_min[GFR_WAVES];
    __shared__ SmState s_st;
    // this launch's mode and bucket from the previous launch's words
    {
        const unsigned long long *pf = a.flags + (size_t)((L & 1) ^ 1) * G;
        uint32_t bits = 0, mn = 0xFFFFFFFFu;
        for (uint32_t i = threadIdx.x; i < G; i += GFR_BLOCK) {
            const unsigned long long f = pf[i];
            bits |= (uint32_t)f;
            mn = min(mn, (uint32_t)(f >> 32));
        }
        bits = wave_or_u32(bits);
        mn = wave_min_u32(mn);
        if (lane == 0) {
            s_bits[wave] = bits;
            s_min[wave] = mn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < GFR_WAVES; ++w) {
                bits |= s_bits[w];
                mn = min(mn, s_min[w]);
            }
            const SmState p = a.st[(L & 1) ^ 1];
            // far marks left after the previous launch: a split examined
            // every older one, so only its kept and new ones remain
            const uint32_t far_any = (p.mode == SM_SPLIT ? 0u : p.far_any) | ((bits & SMF_FAR) ? 1u : 0u);
            const uint32_t far_min = min(p.mode == SM_SPLIT ? 0xFFFFFFFFu : p.far_min, mn);
            SmState st;
            if (p.mode == SM_DONE) {
                st = p;
            } else if (bits & SMF_NEAR) {
                st = SmState{SM_RELAX, p.hi, far_any, far_min};
            } else if (far_any) {
                // next bucket: the smallest far distance falls inside it
                const unsigned long long d = a.delta;
                const unsigned long long nh = ((unsigned long long)far_min / d + 1ull) * d;
                st = SmState{SM_SPLIT, nh > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)nh, far_any, far_min};
            } else {
                st = SmState{SM_DONE, p.hi, 0u, 0xFFFFFFFFu};
            }
            s_st = st;
            if (blockIdx.x == 0) {
                a.st[L & 1] = st;
                if (st.mode == SM_DONE) {
                    a.ctl->iter = (uint32_t)L;
                    a.ctl->done = 1u;
                } else if (st.mode == SM_SPLIT) {
                    a.ctl->splits += 1u;
                }
            }
        }
        __syncthreads();
    }
    const SmState st = s_st;
    unsigned long long *myflag = a.flags + (size_t)(L & 1) * G + blockIdx.x;
    if (st.mode == SM_DONE) {
        if (threadIdx.x == 0) *myflag = 0xFFFFFFFFull << 32;
        return;
    }
    const uint32_t hi = st.hi;
    const uint32_t lo = a.st[(L & 1) ^ 1].hi;   // previous bucket bound (splits drop marks below it)
    uint8_t *cur = st.mode == SM_RELAX ? a.mk[L & 1] : a.far;
    uint8_t *nxt = a.mk[(L & 1) ^ 1];
    constexpr int SM_LIST = GFR_BLOCK * 16;
    __shared__ int32_t s_v[SM_LIST];
    __shared__ uint32_t s_cnt;
    uint32_t bits = 0, fmin = 0xFFFFFFFFu;
    uint32_t nent = 0, nrel = 0, nimp = 0, nfar = 0;
    bool ovf = false;
    const size_t nchunks = ((size_t)a.n + 15) / 16;
    for (size_t c0 = (size_t)blockIdx.x * GFR_BLOCK; c0 < nchunks; c0 += (size_t)G * GFR_BLOCK) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const size_t ci = c0 + threadIdx.x;
        if (ci < nchunks) {
            uint4 *p = (uint4 *)(cur + ci * 16);
            const uint4 w = *p;
            if ((w.x | w.y | w.z | w.w) != 0u) {
                const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
                if (st.mode == SM_RELAX) {
                    *p = make_uint4(0u, 0u, 0u, 0u);   // consumed
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if ((ws[j >> 2] >> (8 * (j & 3))) & 0xFFu) s_v[atomicAdd(&s_cnt, 1u)] = (int32_t)(ci * 16 + j);
                } else {
                    // split: inside the bucket -> relax now; beyond -> keep;
                    // below the previous bound -> relaxed since, dropped.
                    // Marks leave by byte stores: relaxations of this launch
                    // set far marks in the same array (a kept mark is never
                    // rewritten, and a cleared vertex, whose distance is below
                    // the bucket bound, can only gain a near mark)
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        if ((ws[j >> 2] >> (8 * (j & 3))) & 0xFFu) {
                            const int32_t v = (int32_t)(ci * 16 + j);
                            const uint32_t d = a.dist[v];
                            if (d >= hi) {
                                bits |= SMF_FAR;
                                fmin = min(fmin, d);
                            } else {
                                cur[v] = 0;
                                if (d >= lo) s_v[atomicAdd(&s_cnt, 1u)] = v;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t cnt = s_cnt;   // at most 16 per thread: fits SM_LIST
        nent += threadIdx.x < cnt ? (cnt - threadIdx.x + GFR_BLOCK - 1) / GFR_BLOCK : 0u;
        for (uint32_t i = threadIdx.x; i < cnt; i += GFR_BLOCK) {
            const int32_t v = s_v[i];   // only vertices < n are ever marked
            const uint32_t du = a.dist[v];
            const int32_t e1 = a.R[v + 1];
            for (int32_t e = a.R[v]; e < e1; e += 8) {
                int32_t u[8];
                uint32_t w[8], d[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int32_t ek = min(e + k, e1 - 1);
                    u[k] = a.C[ek];
                    w[k] = a.W[ek];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) d[k] = a.dist[u[k]];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (e + k >= e1) continue;
                    ++nrel;
                    const unsigned long long nd64 = (unsigned long long)du + w[k];
                    if (nd64 >= 0xFFFFFFFFull) {
                        ovf = true;
                        continue;
                    }
                    const uint32_t nd = (uint32_t)nd64;
                    if (nd < d[k]) {
                        // non-returning: the mark follows the pre-check (a
                        // superset of the true improvements)
                        atomicMin(a.dist + u[k], nd);
                        ++nimp;
                        if (nd < hi) {
                            nxt[u[k]] = 1;
                            bits |= SMF_NEAR;
                        } else {
                            a.far[u[k]] = 1;
                            bits |= SMF_FAR;
                            fmin = min(fmin, nd);
                            ++nfar;
                        }
                    }
                }
            }
        }
        __syncthreads();   // the list is reused by the next round
    }
    // per-group word for the next launch, counters, unfit sums
    bits = wave_or_u32(bits);
    fmin = wave_min_u32(fmin);
    nent = wave_sum_u32(nent);
    nrel = wave_sum_u32(nrel);
    nimp = wave_sum_u32(nimp);
    nfar = wave_sum_u32(nfar);
    __shared__ uint32_t s_c[4][GFR_WAVES];
    if (lane == 0) {
        s_bits[wave] = bits;
        s_min[wave] = fmin;
        s_c[0][wave] = nent;
        s_c[1][wave] = nrel;
        s_c[2][wave] = nimp;
        s_c[3][wave] = nfar;
    }
    ovf = __syncthreads_or((int)ovf) != 0;
    if (threadIdx.x == 0) {
        uint32_t t[4] = {0u, 0u, 0u, 0u};
        for (int w = 0; w < GFR_WAVES; ++w) {
            bits |= s_bits[w];
            fmin = min(fmin, s_min[w]);
            for (int k = 0; k < 4; ++k) t[k] += s_c[k][w];
        }
        *myflag = ((unsigned long long)fmin << 32) | bits;
        if (ovf) a.ctl->unfit = 1u;
        if (t[0]) atomicAdd(&a.ctl->near_entries, (unsigned long long)t[0]);
        if (t[1]) atomicAdd(&a.ctl->relaxed, (unsigned long long)t[1]);
        if (t[2]) atomicAdd(&a.ctl->improvements, (unsigned long long)t[2]);
        if (t[3]) atomicAdd(&a.ctl->far_entries, (unsigned long long)t[3]);
    }
}

static void run_sssp_marks(Ctx &c, Graph &g, int32_t src, uint32_t *dist, hipStream_t s, uint32_t delta)
{
    const int32_t n = g.n;
    const size_t nb = ((size_t)n + 15) / 16 * 16;
    const int G = grid_blocks(c, 4);
    c.arena.reserve(3 * al256(nb) + al256(16ull * G) + al256(2 * sizeof(SmState)) + al256(sizeof(SmCtl)) + al256(4));
    SmArgs a;
    memset(&a, 0, sizeof a);
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.W = g.W.as<uint32_t>();
    a.n = n;
    a.dist = dist;
    a.mk[0] = c.arena.take<uint8_t>(nb);
    a.mk[1] = c.arena.take<uint8_t>(nb);
    a.far = c.arena.take<uint8_t>(nb);
    a.flags = c.arena.take<unsigned long long>(2ull * G);
    a.st = c.arena.take<SmState>(2);
    a.ctl = c.arena.take<SmCtl>(1);
    uint32_t *unfit_flag = c.arena.take<uint32_t>(1);
    a.delta = delta;
    fill_u32(dist, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.mk[0], 0u, nb / 4, s);
    fill_u32(a.mk[1], 0u, nb / 4, s);
    fill_u32(a.far, 0u, nb / 4, s);
    hipLaunchKernelGGL(sssp_marks_init, dim3((G + 255) / 256), dim3(256), 0, s, a, src, (uint32_t)G);
    GFR_LAUNCH_CHECK();
    int32_t level = 0;
    auto launch = [&]() {
        c.ktimer.run("sssp_mark_level", s, [&]() {
            hipLaunchKernelGGL(sssp_mark_level, dim3(G), dim3(GFR_BLOCK), 0, s, a, level);
        });
        ++level;
    };
    const int64_t cap = 64ll * n + 1024;
    const int32_t launched = run_until_done(c, &a.ctl->done, 1u, g.iter_hint() + 2, cap, s, launch);
    SmCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(SmCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(SmCtl));
    if (h.unfit) sssp_check_unfit(c, g, dist, unfit_flag, s);
    c.stats.v["iterations"] += h.iter;
    c.stats.v["relaxations"] += (double)h.relaxed;
    c.stats.v["edges_inspected"] += (double)h.relaxed;
    c.stats.v["splits"] += h.splits;
    c.stats.v["near_entries"] += (double)h.near_entries;
    c.stats.v["improvements"] += (double)h.improvements;
    c.stats.v["far_entries"] += (double)h.far_entries;
    c.stats.v["delta"] = delta;
    c.stats.v["launches"] += launched;
    c.stats.v["solves"] += 1.0;
    g.sssp_iter_hint.store((int32_t)h.iter, std::memory_order_relaxed);
}

void run_sssp(Ctx &c, Graph &g, int32_t src, uint32_t *dist, hipStream_t s)
{
    if (!g.weighted) fail(GFR_E_INVALID, "sssp: graph was loaded without weights");
    const int32_t n = g.n;
    const uint32_t chunk = (uint32_t)c.opt.advance_chunk;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    const uint32_t delta = c.opt.sssp_delta > 0 ? (uint32_t)c.opt.sssp_delta : sssp_auto_delta(g, c.opt.sssp_delta_factor);
    // mark-byte iterations on request (sssp.frontier 2); auto keeps the queue,
    // which takes fewer iterations on the 4096^2 lattice (241 against 366 at
    // the same bucket width) and is faster there
    const int fr = c.opt.sssp_frontier;
    if (fr == 2) {
        run_sssp_marks(c, g, src, dist, s, delta);
        return;
    }
    const int G = grid_blocks(c, 8);   // eight work-groups per CU fit at the default chunk
    const CompactGeom cg = compact_geom(nwords, c.num_cu);
    size_t need = 2 * al256(nwords * 32ull) + 3 * al256(4ull * n) + al256(4 * nparts) + al256(8ull * G) +
                  al256(16ull * cg.blocks) + al256(sizeof(SsspCtl)) + al256(4) + al256(4ull * nwords);
    c.arena.reserve(need);
    SsspArgs a;
    memset(&a, 0, sizeof a);   // padding too: the bytes key the captured steps
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.W = g.W.as<uint32_t>();
    a.n = n;
    a.nwords = nwords;
    a.dist = dist;
    a.near = c.arena.take<uint8_t>(32ull * nwords);
    a.far = c.arena.take<uint8_t>(32ull * nwords);
    a.q.v = c.arena.take<int32_t>(n);
    a.q.off = c.arena.take<uint32_t>(n);
    a.q.row = c.arena.take<int32_t>(n);
    a.q.part = c.arena.take<int32_t>(nparts);
    a.part = c.arena.take<uint32_t>(2ull * G);
    a.fbits = c.arena.take<uint32_t>(nwords);
    a.full = g.full;
    a.full_nf = (uint32_t)g.full_nf;
    a.full_mf = (uint32_t)g.m;
    unsigned long long *status = c.arena.take<unsigned long long>(2ull * cg.blocks);
    a.ctl = c.arena.take<SsspCtl>(1);
    uint32_t *unfit_flag = c.arena.take<uint32_t>(1);

    fill_u32(dist, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.near, 0u, 8ull * nwords, s);
    fill_u32(a.far, 0u, 8ull * nwords, s);
    fill_u32(status, 0u, 4ull * cg.blocks, s);
    hipLaunchKernelGGL(sssp_init, dim3(1), dim3(GFR_BLOCK), 0, s, a, src, chunk, delta, (float)c.opt.sssp_pull_alpha);
    GFR_LAUNCH_CHECK();

    SsspMarks marks{a, (uint32_t)G};
    const bool pull = c.opt.sssp_pull_alpha > 0;   // direction-optimizing iterations
    auto launch = [&]() {
        c.ktimer.run("sssp_relax", s, [&]() {
            switch (chunk) {
            case 256: hipLaunchKernelGGL(sssp_relax<256>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 512: hipLaunchKernelGGL(sssp_relax<512>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 1024: hipLaunchKernelGGL(sssp_relax<1024>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            case 2048: hipLaunchKernelGGL(sssp_relax<2048>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            default: hipLaunchKernelGGL(sssp_relax<4096>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
            }
        });
        if (pull)
            c.ktimer.run("sssp_pull", s, [&]() {
                hipLaunchKernelGGL(sssp_pull<GATHER_CH>, dim3(G), dim3(GFR_BLOCK), 0, s, a);
            });
        c.ktimer.run("sssp_compact", s, [&]() {
            hipLaunchKernelGGL(compact_kernel<SsspMarks>, dim3(cg.blocks), dim3(GFR_BLOCK), 0, s, a.R, n, nwords,
                               cg.wpt, marks, a.q, chunk, status, &a.ctl->parity, &a.ctl->err);
        });
    };
    // every iteration relaxes or splits; the loop is bounded well below this cap
    const int64_t cap = 64ll * n + 1024;
    StepKey key("sssp");
    key.add(a).add(G).add(cg).add(chunk).add(status).add(pull);
    const int32_t launched = run_until_done(c, &a.ctl->mode, SS_DONE, g.iter_hint() + 1, cap, s, launch, &key);
    SsspCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(SsspCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(SsspCtl));
    if (h.err) fail(GFR_E_DEVICE, "sssp: frontier compaction look-back timed out");
    if (h.unfit) sssp_check_unfit(c, g, dist, unfit_flag, s);
    c.stats.v["iterations"] += h.iter;
    c.stats.v["relaxations"] += (double)h.relaxed;
    c.stats.v["edges_inspected"] += (double)h.relaxed;
    c.stats.v["splits"] += h.splits;
    c.stats.v["near_entries"] += (double)h.near_entries;
    c.stats.v["improvements"] += (double)h.improvements;
    c.stats.v["far_entries"] += (double)h.far_entries;
    c.stats.v["pull_iterations"] += h.pull_iters;
    c.stats.v["delta"] = delta;
    c.stats.v["launches"] += launched;
    c.stats.v["solves"] += 1.0;
    g.sssp_iter_hint.store((int32_t)h.iter, std::memory_order_relaxed);
}

}  // namespace gfr
