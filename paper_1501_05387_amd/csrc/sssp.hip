// sssp.hip -- single-source shortest paths with a near/far priority queue
// (Sec. 4.1 Algorithm 1 for the advance/filter structure, Sec. 4.5 "Priority
// Queue" for the near/far split, Sec. 5.2).
//
// Each iteration is one kernel launch:
//  RELAX  advance over the near queue with the same load-balanced edge chunks
//         as BFS; each edge does atomicMin(dist[v], dist[u] + w) and, if it
//         improved v, the filter is fused in: v is claimed in a per-iteration
//         bitmap (the bitmap-flag dedup of Sec. 5.2) and appended to the next
//         near queue if its new distance is below the bucket bound, otherwise
//         claimed in the far bitmap and appended to the far queue.
//  SPLIT  when the near queue runs dry the bucket advances by delta and the far
//         queue is split: settled entries are dropped, entries inside the new
//         bucket move to near, the rest stay far (Sec. 4.5).
// The last work-group of every launch updates the device control block, so
// iterations are enqueued speculatively by the host.
//
// Claim bitmaps are rotated by iteration parity: iteration i builds queue i+1
// with bitmap (i+1)&1 and wipes, word by word, the claims of queue i in bitmap
// i&1 (every set bit there belongs to queue i, so whole-word stores are safe).
#include "device.h"
#include "engine.h"

namespace gfr {

enum : uint32_t { SS_RELAX = 0, SS_SPLIT = 1, SS_DONE = 2 };

struct SsspCtl {
    unsigned long long next;     // packed counter of the near queue being built
    unsigned long long relaxed;  // edges relaxed so far
    uint32_t mode;               // SS_* (first word read back by the host)
    uint32_t nf, mf;             // entries / edges of the current near queue
    uint32_t cur;                // parity of the current near queue
    uint32_t iter;               // iteration counter
    uint32_t arrive;
    uint32_t far_n;              // entries of far[far_cur]
    uint32_t far_next_n;         // entries kept by a split
    uint32_t far_cur;
    uint32_t lo, hi;             // current bucket [lo, hi)
    uint32_t delta;
    uint32_t min_kept;           // smallest distance left in far by a split
    uint32_t overflow;
    uint32_t splits;
};

struct SsspArgs {
    const int32_t *R;
    const int32_t *C;
    const uint32_t *W;
    int32_t n;
    uint32_t nwords;
    uint32_t *dist;
    uint32_t *nb[2];
    uint32_t *fbm;
    int32_t *far[2];
    FrontierQ q[2];
    SsspCtl *ctl;
};

template <int CH>
__global__ __launch_bounds__(GFR_BLOCK) void sssp_step(SsspArgs a)
{
    SsspCtl *ctl = a.ctl;
    const uint32_t mode = ctl->mode;
    if (mode == SS_DONE) return;
    const uint32_t iter = ctl->iter, cur = ctl->cur;
    const FrontierQ qin = a.q[cur], qout = a.q[cur ^ 1];
    uint32_t *nb_in = a.nb[iter & 1], *nb_out = a.nb[(iter + 1) & 1];
    const uint32_t lo = ctl->lo, hi = ctl->hi;
    const uint32_t gtid = blockIdx.x * GFR_BLOCK + threadIdx.x, gstride = gridDim.x * GFR_BLOCK;

    if (mode == SS_RELAX) {
        const uint32_t nf = ctl->nf, mf = ctl->mf;
        for (uint32_t i = gtid; i < nf; i += gstride) nb_in[qin.v[i] >> 5] = 0u;

        __shared__ uint32_t s_off[CH + 1];
        __shared__ int32_t s_row[CH + 1];
        __shared__ uint32_t s_du[CH + 1];
        const uint32_t nchunks = (mf + CH - 1) / CH;
        int32_t *farq = a.far[ctl->far_cur];
        bool ovf = false;
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
                s_du[i] = a.dist[qin.v[s + i]];
            }
            __syncthreads();
#pragma unroll 1
            for (uint32_t k = 0; k < (uint32_t)CH; k += GFR_BLOCK) {
                const uint32_t e = e0 + k + threadIdx.x;
                bool near_new = false, far_new = false;
                int32_t v = 0, rv = 0;
                uint32_t dv = 0;
                if (e < e1) {
                    const int i = upper_index(s_off, 0, cnt - 1, e);
                    const int32_t idx = s_row[i] + (int32_t)(e - s_off[i]);
                    v = a.C[idx];
                    const unsigned long long nd64 = (unsigned long long)s_du[i] + a.W[idx];
                    if (nd64 >= 0xFFFFFFFFull) {
                        ovf = true;
                    } else {
                        const uint32_t nd = (uint32_t)nd64;
                        if (nd < a.dist[v] && nd < atomicMin(a.dist + v, nd)) {
                            const uint32_t bit = 1u << (v & 31);
                            if (nd < hi) {
                                near_new = !(atomicOr(nb_out + (v >> 5), bit) & bit);
                                if (near_new) {
                                    rv = a.R[v];
                                    dv = (uint32_t)(a.R[v + 1] - rv);
                                }
                            } else {
                                far_new = !(atomicOr(a.fbm + (v >> 5), bit) & bit);
                            }
                        }
                    }
                }
                wave_enqueue(near_new, v, dv, rv, &ctl->next, qout, CH);
                wave_append(far_new, v, &ctl->far_n, farq);
            }
        }
        if (ovf) ctl->overflow = 1u;
    } else {  // SS_SPLIT with bucket [lo, hi)
        const uint32_t fn = ctl->far_n;
        const int32_t *fin = a.far[ctl->far_cur];
        int32_t *fout = a.far[ctl->far_cur ^ 1];
        uint32_t mk = 0xFFFFFFFFu;
        for (uint32_t base = blockIdx.x * GFR_BLOCK; base < fn; base += gstride) {
            const uint32_t i = base + threadIdx.x;
            bool to_near = false, keep = false;
            int32_t v = 0, rv = 0;
            uint32_t dv = 0;
            if (i < fn) {
                v = fin[i];
                const uint32_t d = a.dist[v];
                const uint32_t bit = 1u << (v & 31);
                if (d < hi) {
                    atomicAnd(a.fbm + (v >> 5), ~bit);
                    if (d >= lo) {
                        to_near = !(atomicOr(nb_out + (v >> 5), bit) & bit);
                        if (to_near) {
                            rv = a.R[v];
                            dv = (uint32_t)(a.R[v + 1] - rv);
                        }
                    }
                } else {
                    keep = true;
                    mk = min(mk, d);
                }
            }
            wave_enqueue(to_near, v, dv, rv, &ctl->next, qout, CH);
            wave_append(keep, v, &ctl->far_next_n, fout);
        }
        mk = wave_min_u32(mk);
        if (lane_id() == 0 && mk != 0xFFFFFFFFu) atomicMin(&ctl->min_kept, mk);
    }

    if (last_block_arrives(&ctl->arrive) && threadIdx.x == 0) {
        const unsigned long long nx = atomicAdd(&ctl->next, 0ull);
        const uint32_t nf2 = (uint32_t)(nx >> 32), mf2 = (uint32_t)nx;
        const uint32_t D = ctl->delta;
        if (mode == SS_RELAX) {
            ctl->relaxed += ctl->mf;
        } else {
            ctl->far_n = atomicAdd(&ctl->far_next_n, 0u);
            ctl->far_next_n = 0u;
            ctl->far_cur ^= 1u;
            ctl->splits += 1u;
        }
        const uint32_t far_n = atomicAdd(&ctl->far_n, 0u);
        uint32_t nm;
        if (ctl->overflow) {
            nm = SS_DONE;
        } else if (nf2 > 0) {
            nm = SS_RELAX;
        } else if (far_n > 0) {
            nm = SS_SPLIT;
            unsigned long long nhi = (unsigned long long)hi + D;
            if (mode == SS_SPLIT) {
                // nothing fell into the bucket: jump to the one holding the smallest far distance
                const unsigned long long mk = ctl->min_kept;
                const unsigned long long j = (mk / D + 1ull) * D;
                if (j > nhi) nhi = j;
            }
            ctl->lo = hi;
            ctl->hi = nhi > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)nhi;
        } else {
            nm = SS_DONE;
        }
        ctl->min_kept = 0xFFFFFFFFu;
        ctl->nf = nf2;
        ctl->mf = mf2;
        ctl->next = 0ull;
        ctl->cur = cur ^ 1u;
        ctl->iter = iter + 1u;
        ctl->mode = nm;
    }
}

__global__ void sssp_init(SsspArgs a, int32_t src, uint32_t chunk, uint32_t delta)
{
    const int32_t rs = a.R[src], deg = a.R[src + 1] - rs;
    if (threadIdx.x == 0) {
        SsspCtl *ctl = a.ctl;
        a.dist[src] = 0u;
        a.q[0].v[0] = src;
        a.q[0].off[0] = 0;
        a.q[0].row[0] = rs;
        ctl->next = 0ull;
        ctl->relaxed = 0ull;
        ctl->nf = 1;
        ctl->mf = (uint32_t)deg;
        ctl->cur = 0;
        ctl->iter = 0;
        ctl->arrive = 0;
        ctl->far_n = ctl->far_next_n = 0;
        ctl->far_cur = 0;
        ctl->lo = 0;
        ctl->hi = delta;
        ctl->delta = delta;
        ctl->min_kept = 0xFFFFFFFFu;
        ctl->overflow = 0;
        ctl->splits = 0;
        ctl->mode = deg == 0 ? SS_DONE : SS_RELAX;
    }
    for (uint32_t c = threadIdx.x; (uint64_t)c * chunk < (uint64_t)deg; c += blockDim.x) a.q[0].part[c] = 0;
}

uint32_t sssp_auto_delta(const Graph &g)
{
    double d = g.mean_w * 2.0;
    if (d < 1.0) d = 1.0;
    if (d > 1.0e9) d = 1.0e9;
    return (uint32_t)d;
}

void run_sssp(Ctx &c, Graph &g, int32_t src, uint32_t *dist, hipStream_t s)
{
    if (!g.weighted) fail(GFR_E_INVALID, "sssp: graph was loaded without weights");
    const int32_t n = g.n;
    const uint32_t chunk = (uint32_t)c.opt.advance_chunk;
    const uint32_t nwords = (uint32_t)(((int64_t)n + 63) / 64) * 2u;
    const size_t nparts = (size_t)(g.m / chunk) + 2;
    const uint32_t delta = c.opt.sssp_delta > 0 ? (uint32_t)c.opt.sssp_delta : sssp_auto_delta(g);
    size_t need = 3 * al256(nwords * 4ull) + 2 * al256(4ull * n) +
                  2 * (3 * al256(4ull * n) + al256(4 * nparts)) + al256(sizeof(SsspCtl));
    c.arena.reserve(need);
    SsspArgs a;
    a.R = g.R.as<int32_t>();
    a.C = g.C.as<int32_t>();
    a.W = g.W.as<uint32_t>();
    a.n = n;
    a.nwords = nwords;
    a.dist = dist;
    a.nb[0] = c.arena.take<uint32_t>(nwords);
    a.nb[1] = c.arena.take<uint32_t>(nwords);
    a.fbm = c.arena.take<uint32_t>(nwords);
    a.far[0] = c.arena.take<int32_t>(n);
    a.far[1] = c.arena.take<int32_t>(n);
    for (int i = 0; i < 2; ++i) {
        a.q[i].v = c.arena.take<int32_t>(n);
        a.q[i].off = c.arena.take<uint32_t>(n);
        a.q[i].row = c.arena.take<int32_t>(n);
        a.q[i].part = c.arena.take<int32_t>(nparts);
    }
    a.ctl = c.arena.take<SsspCtl>(1);

    fill_u32(dist, 0xFFFFFFFFu, (size_t)n, s);
    fill_u32(a.nb[0], 0u, nwords, s);
    fill_u32(a.nb[1], 0u, nwords, s);
    fill_u32(a.fbm, 0u, nwords, s);
    hipLaunchKernelGGL(sssp_init, dim3(1), dim3(GFR_BLOCK), 0, s, a, src, chunk, delta);
    GFR_LAUNCH_CHECK();

    const int G = grid_blocks(c, 4);
    auto launch = [&]() { c.ktimer.run("sssp_step", s, [&]() {
        switch (chunk) {
        case 256: hipLaunchKernelGGL(sssp_step<256>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 512: hipLaunchKernelGGL(sssp_step<512>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 1024: hipLaunchKernelGGL(sssp_step<1024>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        case 2048: hipLaunchKernelGGL(sssp_step<2048>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        default: hipLaunchKernelGGL(sssp_step<4096>, dim3(G), dim3(GFR_BLOCK), 0, s, a); break;
        }
    }); };
    // every iteration relaxes or splits; a vertex can be re-improved at most
    // once per distinct distance, so the loop is bounded well below this cap
    const int64_t cap = 64ll * n + 1024;
    const int32_t launched = run_until_done(c, &a.ctl->mode, SS_DONE, g.sssp_iter_hint + 1, cap, s, launch);
    SsspCtl h;
    GFR_HIP(hipMemcpyAsync(c.pinned, a.ctl, sizeof(SsspCtl), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    memcpy(&h, c.pinned, sizeof(SsspCtl));
    if (h.overflow) fail(GFR_E_INVALID, "sssp: a path weight does not fit below 0xFFFFFFFF");
    c.stats.v["iterations"] = h.iter;
    c.stats.v["relaxations"] = (double)h.relaxed;
    c.stats.v["edges_inspected"] = (double)h.relaxed;
    c.stats.v["splits"] = h.splits;
    c.stats.v["delta"] = delta;
    c.stats.v["launches"] = launched;
    g.sssp_iter_hint = (int32_t)h.iter;
}

}  // namespace gfr
