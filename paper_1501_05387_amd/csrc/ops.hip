// ops.hip -- the frontier operators on their own, for callers that compose
// their own traversals (Sec. 3-4: advance and filter are the two operators
// every primitive is built from).
//
//   advance  a vertex frontier (any order, duplicates allowed) becomes its
//            edge frontier: for every entry u, in frontier order, every edge
//            e of u in CSR order, as (u, e, C[e]).  The entries' degrees are
//            scanned into output offsets (the scan of Sec. 4.4), the entries
//            with edges become a chunked frontier queue, and the
//            load-balanced advance writes each edge at its offset, so the
//            output order is exactly the sequential one.  An edge frontier
//            (Sec. 4.1 lets advance start from edges as well) is first
//            gathered to the edges' far ends; each output then carries the
//            input edge in place of u.
//   filter   a list of vertices (duplicates allowed) becomes the ascending
//            list of the distinct vertices not excluded by a byte mask:
//            items leave a mark byte (idempotent stores, Sec. 4.5), and a
//            scan over the marks compacts them in vertex order.
//   scan     the exact exclusive prefix sum (uint64) of a uint32 array: the
//            scan that turns degrees into output offsets (Sec. 4.4), alone.
//   split    the near/far split of a frontier (Sec. 4.5, priority queue):
//            items whose distance is below a threshold go to the near list,
//            the others to the far list, both in input order (one scan of
//            the pair (near, far) gives every item its slot).
//
// Both scans run in three launches: per-tile totals, one work-group scanning
// the tile totals, and a pass that recomputes each tile's prefix and writes.
// Each thread owns SCAN_EPT consecutive elements, so every write lands at
// its exclusive prefix.
#include <string.h>

#include <algorithm>
#include <string>

#include "compact.h"
#include "engine.h"

namespace gfr {

constexpr int SCAN_EPT = 8;
constexpr int64_t SCAN_TILE = (int64_t)GFR_BLOCK * SCAN_EPT;

struct P2 {
    unsigned long long a, b;   // advance: edges, queue entries; filter: unused, list entries
};

__device__ __forceinline__ P2 block_excl_scan_p2(P2 x, P2 *total)
{
    unsigned long long ta, tb;
    P2 r;
    r.a = block_excl_scan_u64(x.a, &ta);
    r.b = block_excl_scan_u64(x.b, &tb);
    total->a = ta;
    total->b = tb;
    return r;
}

// per-tile totals
template <class Val>
__global__ __launch_bounds__(GFR_BLOCK) void scan_reduce(Val val, int64_t count, P2 *totals)
{
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    P2 s{0, 0};
    for (int64_t i = t0 + threadIdx.x; i < count && i < t0 + SCAN_TILE; i += GFR_BLOCK) {
        const P2 x = val(i);
        s.a += x.a;
        s.b += x.b;
    }
    P2 tot;
    (void)block_excl_scan_p2(s, &tot);
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// exclusive scan of the tile totals in place (one work-group); grand total at totals[ntiles]
__global__ __launch_bounds__(GFR_BLOCK) void scan_totals(P2 *totals, int64_t ntiles)
{
    P2 carry{0, 0};
    for (int64_t b0 = 0; b0 < ntiles; b0 += GFR_BLOCK) {
        const int64_t i = b0 + threadIdx.x;
        const P2 x = i < ntiles ? totals[i] : P2{0, 0};
        P2 tot;
        const P2 ex = block_excl_scan_p2(x, &tot);
        if (i < ntiles) totals[i] = P2{carry.a + ex.a, carry.b + ex.b};
        carry.a += tot.a;
        carry.b += tot.b;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[ntiles] = carry;
}

// each element with its exclusive prefix
template <class Val, class Emit>
__global__ __launch_bounds__(GFR_BLOCK) void scan_emit(Val val, int64_t count, const P2 *totals, Emit emit)
{
    const int64_t i0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_EPT;
    P2 x[SCAN_EPT];
    P2 s{0, 0};
#pragma unroll
    for (int j = 0; j < SCAN_EPT; ++j) {
        x[j] = i0 + j < count ? val(i0 + j) : P2{0, 0};
        s.a += x[j].a;
        s.b += x[j].b;
    }
    P2 tot;
    const P2 ex = block_excl_scan_p2(s, &tot);
    P2 p{totals[blockIdx.x].a + ex.a, totals[blockIdx.x].b + ex.b};
#pragma unroll
    for (int j = 0; j < SCAN_EPT; ++j) {
        if (i0 + j < count) emit(i0 + j, x[j], p);
        p.a += x[j].a;
        p.b += x[j].b;
    }
}

// ------------------------------------------------------------ advance

struct AdvVal {
    const int32_t *F;
    const int32_t *R;
    __device__ P2 operator()(int64_t i) const
    {
        const int32_t v = F[i];
        const unsigned long long d = (unsigned long long)(R[v + 1] - R[v]);
        return P2{d, d ? 1ull : 0ull};
    }
};

// entries with edges become the queue, tagged with their input item (the
// vertex itself, or the edge it was reached by); part[c] = entry holding edge
// c * CH
struct AdvEmit {
    const int32_t *F;
    const int32_t *T;
    const int32_t *R;
    FrontierQ q;
    __device__ void operator()(int64_t i, P2 x, P2 p) const
    {
        if (!x.a) return;
        const int32_t v = F[i];
        const uint32_t slot = (uint32_t)p.b, off = (uint32_t)p.a, d = (uint32_t)x.a;
        q.v[slot] = T[i];
        q.off[slot] = off;
        q.row[slot] = R[v];
        for (uint32_t c = (off + GATHER_CH - 1) / GATHER_CH; (uint64_t)c * GATHER_CH < (uint64_t)off + d; ++c)
            q.part[c] = (int32_t)slot;
    }
};

// every edge of the queue, written at its offset
__global__ __launch_bounds__(GFR_BLOCK) void advance_emit(FrontierQ q, uint32_t nf, uint32_t mf, const int32_t *C,
                                                          int32_t *out_src, int32_t *out_edge, int32_t *out_dst)
{
    constexpr uint32_t CH = GATHER_CH;
    __shared__ uint32_t s_off[CH + 1];
    __shared__ int32_t s_row[CH + 1];
    __shared__ int32_t s_v[CH + 1];
    const uint32_t nchunks = (mf + CH - 1) / CH;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t e0 = c * CH, e1 = min(e0 + CH, mf);
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
        for (uint32_t p = e0 + threadIdx.x; p < e1; p += GFR_BLOCK) {
            const int i = upper_index(s_off, 0, cnt - 1, p);
            const int32_t e = s_row[i] + (int32_t)(p - s_off[i]);
            if (out_src) out_src[p] = s_v[i];
            if (out_edge) out_edge[p] = e;
            if (out_dst) out_dst[p] = C[e];
        }
    }
}

// far ends of an edge frontier
__global__ void edge_heads(const int32_t *E, int64_t count, const int32_t *C, int32_t *V)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        V[i] = C[E[i]];
}

__global__ void count_out_of_range(const int32_t *x, int64_t count, int32_t n, uint32_t *bad)
{
    uint32_t b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        b += (x[i] < 0 || x[i] >= n) ? 1u : 0u;
    if (b) atomicAdd(bad, b);
}

// Input list on the device (copied there when it is host memory), every id
// checked against [0, n).
static const int32_t *device_list(Ctx &c, const int32_t *list, int64_t count, int32_t n, int32_t *staging,
                                  uint32_t *bad, hipStream_t s, const char *who, const char *what = "vertex")
{
    const int32_t *d = list;
    if (!is_device_ptr(list)) {
        GFR_HIP(hipMemcpyAsync(staging, list, 4ull * count, hipMemcpyHostToDevice, s));
        d = staging;
    }
    fill_u32(bad, 0u, 1, s);
    hipLaunchKernelGGL(count_out_of_range, dim3(grid_blocks(c, 2)), dim3(GFR_BLOCK), 0, s, d, count, n, bad);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, bad, 4, hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    if (c.pinned[0]) fail(GFR_E_INVALID, std::string(who) + ": " + what + " id out of range");
    return d;
}

int64_t run_advance(Ctx &c, Graph &g, const int32_t *frontier, int32_t nf, bool edges, int32_t *out_src,
                    int32_t *out_edge, int32_t *out_dst, int64_t out_cap, hipStream_t s)
{
    const int64_t ntiles = (nf + SCAN_TILE - 1) / SCAN_TILE;
    const int64_t cap = std::min<int64_t>(out_cap, INT32_MAX);
    const size_t nparts = (size_t)(cap / GATHER_CH) + 2;
    c.arena.reserve(2 * al256(4ull * nf) + al256(16ull * (ntiles + 1)) + al256(16) + 3 * al256(4ull * nf) +
                    al256(4 * nparts));
    int32_t *staging = c.arena.take<int32_t>(nf);
    int32_t *heads = c.arena.take<int32_t>(nf);
    P2 *totals = c.arena.take<P2>(ntiles + 1);
    uint32_t *bad = c.arena.take<uint32_t>(4);
    FrontierQ q{c.arena.take<int32_t>(nf), c.arena.take<uint32_t>(nf), c.arena.take<int32_t>(nf),
                c.arena.take<int32_t>(nparts)};
    if (nf == 0) return 0;
    const int32_t *R = g.R.as<int32_t>();
    const int32_t *T, *F;   // tags written as out_src; vertices expanded
    if (edges) {
        T = device_list(c, frontier, nf, (int32_t)g.m, staging, bad, s, "advance_edges", "edge");
        hipLaunchKernelGGL(edge_heads, dim3(grid_blocks(c, 2)), dim3(GFR_BLOCK), 0, s, T, (int64_t)nf,
                           g.C.as<int32_t>(), heads);
        GFR_LAUNCH_CHECK();
        F = heads;
    } else {
        T = F = device_list(c, frontier, nf, g.n, staging, bad, s, "advance");
    }
    hipLaunchKernelGGL(scan_reduce<AdvVal>, dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, AdvVal{F, R}, (int64_t)nf,
                       totals);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(GFR_BLOCK), 0, s, totals, ntiles);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, totals + ntiles, sizeof(P2), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    P2 grand;
    memcpy(&grand, c.pinned, sizeof grand);
    const int64_t total = (int64_t)grand.a;
    if (total > out_cap || total > INT32_MAX) return total;   // the caller reports the capacity error
    hipLaunchKernelGGL((scan_emit<AdvVal, AdvEmit>), dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, AdvVal{F, R},
                       (int64_t)nf, totals, AdvEmit{F, T, R, q});
    if (total > 0)
        hipLaunchKernelGGL(advance_emit, dim3(grid_blocks(c, 4)), dim3(GFR_BLOCK), 0, s, q, (uint32_t)grand.b,
                           (uint32_t)total, g.C.as<int32_t>(), out_src, out_edge, out_dst);
    GFR_LAUNCH_CHECK();
    c.stats.v["edges"] = (double)total;
    c.stats.v["entries_with_edges"] = (double)grand.b;
    return total;
}

// ------------------------------------------------------------- filter

__global__ void mark_items(const int32_t *items, int64_t count, const uint8_t *exclude, uint8_t *mark)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = items[i];
        if (!exclude || !exclude[v]) mark[v] = 1;
    }
}

struct MarkVal {
    const uint8_t *mark;
    __device__ P2 operator()(int64_t i) const { return P2{0ull, mark[i] ? 1ull : 0ull}; }
};

struct ListEmit {
    int32_t *out;
    __device__ void operator()(int64_t i, P2 x, P2 p) const
    {
        if (x.b) out[p.b] = (int32_t)i;
    }
};

int64_t run_filter(Ctx &c, Graph &g, const int32_t *items, int64_t count, const uint8_t *exclude, int32_t *out,
                   int64_t out_cap, hipStream_t s)
{
    const int32_t n = g.n;
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    c.arena.reserve(al256(4ull * count) + al256(16ull * (ntiles + 1)) + al256(16) + al256(4ull * ((n + 3) / 4)) +
                    al256(n));
    int32_t *staging = c.arena.take<int32_t>(count);
    P2 *totals = c.arena.take<P2>(ntiles + 1);
    uint32_t *bad = c.arena.take<uint32_t>(4);
    uint8_t *mark = c.arena.take<uint8_t>(4ull * ((n + 3) / 4));
    if (exclude && !is_device_ptr(exclude)) {
        uint8_t *excl_dev = c.arena.take<uint8_t>(n);
        GFR_HIP(hipMemcpyAsync(excl_dev, exclude, (size_t)n, hipMemcpyHostToDevice, s));
        exclude = excl_dev;
    }
    fill_u32(mark, 0u, (n + 3) / 4, s);
    if (count > 0) {
        const int32_t *X = device_list(c, items, count, n, staging, bad, s, "filter");
        hipLaunchKernelGGL(mark_items, dim3(grid_blocks(c, 2)), dim3(GFR_BLOCK), 0, s, X, count, exclude, mark);
    }
    hipLaunchKernelGGL(scan_reduce<MarkVal>, dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, MarkVal{mark}, (int64_t)n,
                       totals);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(GFR_BLOCK), 0, s, totals, ntiles);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, totals + ntiles, sizeof(P2), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    P2 grand;
    memcpy(&grand, c.pinned, sizeof grand);
    const int64_t kept = (int64_t)grand.b;
    if (kept > out_cap) return kept;   // the caller reports the capacity error
    hipLaunchKernelGGL((scan_emit<MarkVal, ListEmit>), dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, MarkVal{mark},
                       (int64_t)n, totals, ListEmit{out});
    GFR_LAUNCH_CHECK();
    c.stats.v["kept"] = (double)kept;
    return kept;
}

// ------------------------------------------------------------- scan

struct ScanVal {
    const uint32_t *x;
    __device__ P2 operator()(int64_t i) const { return P2{(unsigned long long)x[i], 0ull}; }
};

struct ScanEmit {
    unsigned long long *out;
    __device__ void operator()(int64_t i, P2, P2 p) const { out[i] = p.a; }
};

uint64_t run_scan(Ctx &c, const uint32_t *in, int64_t count, unsigned long long *out, hipStream_t s)
{
    const int64_t ntiles = (count + SCAN_TILE - 1) / SCAN_TILE;
    c.arena.reserve(al256(4ull * count) + al256(16ull * (ntiles + 1)));
    uint32_t *staging = c.arena.take<uint32_t>(count);
    P2 *totals = c.arena.take<P2>(ntiles + 1);
    if (count == 0) return 0;
    const uint32_t *X = in;
    if (!is_device_ptr(in)) {
        GFR_HIP(hipMemcpyAsync(staging, in, 4ull * count, hipMemcpyHostToDevice, s));
        X = staging;
    }
    hipLaunchKernelGGL(scan_reduce<ScanVal>, dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, ScanVal{X}, count, totals);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(GFR_BLOCK), 0, s, totals, ntiles);
    hipLaunchKernelGGL((scan_emit<ScanVal, ScanEmit>), dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, ScanVal{X},
                       count, totals, ScanEmit{out});
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, totals + ntiles, sizeof(P2), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    P2 grand;
    memcpy(&grand, c.pinned, sizeof grand);
    return grand.a;
}

// ------------------------------------------------------------- split

struct SplitVal {
    const int32_t *X;
    const uint32_t *dist;
    uint32_t thr;
    __device__ P2 operator()(int64_t i) const
    {
        const bool nr = dist[X[i]] < thr;
        return P2{nr ? 1ull : 0ull, nr ? 0ull : 1ull};
    }
};

struct SplitEmit {
    const int32_t *X;
    int32_t *near, *far;
    __device__ void operator()(int64_t i, P2 x, P2 p) const
    {
        if (x.a) near[p.a] = X[i];
        else far[p.b] = X[i];
    }
};

void run_split(Ctx &c, Graph &g, const int32_t *items, int64_t count, const uint32_t *dist, uint32_t threshold,
               int32_t *near, int32_t *far, int64_t out_cap, int64_t *n_near, int64_t *n_far, hipStream_t s)
{
    const int32_t n = g.n;
    const int64_t ntiles = (count + SCAN_TILE - 1) / SCAN_TILE;
    c.arena.reserve(al256(4ull * count) + al256(16ull * (ntiles + 1)) + al256(16) + al256(4ull * n));
    int32_t *staging = c.arena.take<int32_t>(count);
    P2 *totals = c.arena.take<P2>(ntiles + 1);
    uint32_t *bad = c.arena.take<uint32_t>(4);
    uint32_t *dist_dev = c.arena.take<uint32_t>(n);
    *n_near = *n_far = 0;
    if (count == 0) return;
    const int32_t *X = device_list(c, items, count, n, staging, bad, s, "split");
    const uint32_t *D = dist;
    if (!is_device_ptr(dist)) {
        GFR_HIP(hipMemcpyAsync(dist_dev, dist, 4ull * n, hipMemcpyHostToDevice, s));
        D = dist_dev;
    }
    const SplitVal val{X, D, threshold};
    hipLaunchKernelGGL(scan_reduce<SplitVal>, dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, val, count, totals);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(GFR_BLOCK), 0, s, totals, ntiles);
    GFR_LAUNCH_CHECK();
    GFR_HIP(hipMemcpyAsync(c.pinned, totals + ntiles, sizeof(P2), hipMemcpyDeviceToHost, s));
    GFR_HIP(hipStreamSynchronize(s));
    P2 grand;
    memcpy(&grand, c.pinned, sizeof grand);
    *n_near = (int64_t)grand.a;
    *n_far = (int64_t)grand.b;
    if (*n_near > out_cap || *n_far > out_cap) return;   // the caller reports the capacity error
    hipLaunchKernelGGL((scan_emit<SplitVal, SplitEmit>), dim3((uint32_t)ntiles), dim3(GFR_BLOCK), 0, s, val, count,
                       totals, SplitEmit{X, near, far});
    GFR_LAUNCH_CHECK();
}

}  // namespace gfr
