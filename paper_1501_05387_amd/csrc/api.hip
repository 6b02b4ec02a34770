// api.hip -- the C ABI (include/gfr.h): contexts, resident graphs, argument
// checking, output placement (host or device), and dispatch to the solvers.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"

namespace gfr {

void fail(gfr_status code, const std::string &msg) { throw Error{code, msg}; }

Graph &get_graph(Ctx &c, gfr_graph h)
{
    auto it = c.graphs.find(h);
    if (it == c.graphs.end()) fail(GFR_E_NOT_FOUND, "unknown graph handle " + std::to_string(h));
    return *it->second;
}

bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

int grid_blocks(const Ctx &c, int per_cu) { return c.num_cu * per_cu; }

int resident_grid(const Ctx &c, const void *kernel, int per_cu)
{
    if (per_cu > 0) return c.num_cu * per_cu;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, GFR_BLOCK, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 4;
    }
    return c.num_cu * nb;
}

// Scratch of gfr_bfs_noalloc: one fixed array per device (the code object's
// copy on that device), never allocated or freed by the library.  Host code
// must not use the array's name as an address: it is a host-side stand-in.
// The device address is looked up once per device, with that device current,
// and kept here.
static __device__ __align__(256) unsigned char scratch[GFR_NOALLOC_SCRATCH_BYTES];
static std::mutex scratch_mu;
static std::map<int, void *> scratch_addr;

// Device address of `scratch` on `device`, which must be the current device.
static void *noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    auto it = scratch_addr.find(device);
    if (it != scratch_addr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        fail(GFR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    scratch_addr[device] = ptr;
    return ptr;
}

// true if p is device memory of `device`
static bool is_device_ptr_on(const void *p, int device)
{
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice && attr.device == device;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

void fill_u32(void *p, uint32_t value, size_t count, hipStream_t s)
{
    if (count == 0) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, value, count);
    GFR_LAUNCH_CHECK();
}

static bool is_pinned_host(const void *p)
{
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

static void parallel_memcpy(char *dst, const char *src, size_t bytes)
{
    constexpr size_t kSlice = 4u << 20;
    const size_t nt = std::min<size_t>(8, (bytes + kSlice - 1) / kSlice);
    if (nt <= 1) {
        memcpy(dst, src, bytes);
        return;
    }
    const size_t per = (bytes + nt - 1) / nt;
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) {
        const size_t o = t * per, l = o < bytes ? std::min(per, bytes - o) : 0;
        if (l) th.emplace_back([=]() { memcpy(dst + o, src + o, l); });
    }
    memcpy(dst, src, std::min(per, bytes));
    for (auto &x : th) x.join();
}

void copy_to_host(Bounce &b, void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (is_pinned_host(dst)) {
        GFR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        return;
    }
    constexpr size_t kChunk = 32u << 20;
    for (int i = 0; i < 2; ++i) {
        if (!b.buf[i]) GFR_HIP(hipHostMalloc((void **)&b.buf[i], kChunk, hipHostMallocDefault));
        if (!b.ev[i]) GFR_HIP(hipEventCreateWithFlags(&b.ev[i], hipEventDisableTiming));
    }
    const size_t nch = (bytes + kChunk - 1) / kChunk;
    auto len = [&](size_t j) { return std::min(kChunk, bytes - j * kChunk); };
    auto enqueue = [&](size_t j) {
        GFR_HIP(hipMemcpyAsync(b.buf[j & 1], (const char *)src + j * kChunk, len(j), hipMemcpyDeviceToHost, s));
        GFR_HIP(hipEventRecord(b.ev[j & 1], s));
    };
    enqueue(0);
    for (size_t j = 0; j < nch; ++j) {
        // buffer (j+1)&1 was drained by the host copy of chunk j-1 just below
        if (j + 1 < nch) enqueue(j + 1);
        GFR_HIP(hipEventSynchronize(b.ev[j & 1]));
        parallel_memcpy((char *)dst + j * kChunk, b.buf[j & 1], len(j));
    }
}

// Host check of a CSR graph; returns an empty string when it is acceptable.
static std::string check_csr(int32_t n, int64_t m, const int32_t *R, const int32_t *C,
                             const uint32_t *W, uint32_t flags)
{
    (void)W;
    if (n <= 0) return "n must be positive";
    if (m < 0) return "m must be non-negative";
    if (m > (int64_t)INT32_MAX - 1) return "m must be below 2^31-1";
    if (!R || (m > 0 && !C)) return "null CSR array";
    if (R[0] != 0) return "row_offsets[0] must be 0";
    if ((int64_t)R[n] != m) return "row_offsets[n] must equal m";
    for (int32_t i = 0; i < n; ++i)
        if (R[i + 1] < R[i]) return "row_offsets decrease at row " + std::to_string(i);
    for (int64_t e = 0; e < m; ++e)
        if (C[e] < 0 || C[e] >= n) return "column id out of range at entry " + std::to_string(e);
    if (flags & GFR_VALIDATE) {
        for (int32_t u = 0; u < n; ++u) {
            for (int32_t e = R[u]; e < R[u + 1]; ++e) {
                if (C[e] == u) return "self loop at vertex " + std::to_string(u);
                if (e > R[u] && C[e] <= C[e - 1])
                    return "row " + std::to_string(u) + " not strictly increasing (unsorted or duplicate)";
            }
        }
        // symmetry: every (u,v) has (v,u) with the same weight
        for (int32_t u = 0; u < n; ++u) {
            for (int32_t e = R[u]; e < R[u + 1]; ++e) {
                const int32_t v = C[e];
                const int32_t *b = C + R[v], *en = C + R[v + 1];
                const int32_t *f = std::lower_bound(b, en, u);
                if (f == en || *f != u)
                    return "asymmetric: edge " + std::to_string(u) + "->" + std::to_string(v) + " has no reverse";
                if (W && W[f - C] != W[e])
                    return "asymmetric weights on edge " + std::to_string(u) + "-" + std::to_string(v);
            }
        }
    }
    return std::string();
}

// The whole vertex set as a frontier queue, chunked for the gather kernels.
static void build_full_queue(Ctx &c, Graph &g, const int32_t *R)
{
    const int32_t n = g.n;
    std::vector<int32_t> v, row;
    std::vector<uint32_t> off;
    v.reserve(n);
    for (int32_t i = 0; i < n; ++i)
        if (R[i + 1] > R[i]) v.push_back(i);
    const int32_t nf = (int32_t)v.size();
    off.resize(nf);
    row.resize(nf);
    for (int32_t i = 0; i < nf; ++i) {
        off[i] = (uint32_t)R[v[i]];
        row[i] = R[v[i]];
    }
    const size_t nch = (size_t)(g.m + GATHER_CH - 1) / GATHER_CH;
    std::vector<int32_t> part(nch + 1, 0);
    {
        size_t ci = 0;
        for (int32_t i = 0; i < nf && ci < nch; ++i) {
            const uint64_t end = (uint64_t)off[i] + (uint64_t)(R[v[i] + 1] - R[v[i]]);
            while (ci < nch && (uint64_t)ci * GATHER_CH < end) part[ci++] = i;
        }
    }
    const size_t b_v = al256(4ull * std::max(nf, 1)), b_p = al256(4ull * (nch + 1));
    g.full_mem.alloc(3 * b_v + b_p + 256);
    char *base = (char *)g.full_mem.p;
    g.full.v = (int32_t *)base;
    g.full.off = (uint32_t *)(base + b_v);
    g.full.row = (int32_t *)(base + 2 * b_v);
    g.full.part = (int32_t *)(base + 3 * b_v);
    g.full_counts = (uint32_t *)(base + 3 * b_v + b_p);
    uint32_t counts[4] = {(uint32_t)nf, (uint32_t)g.m, 0u, 0u};
    if (nf) {
        GFR_HIP(hipMemcpyAsync(g.full.v, v.data(), 4ull * nf, hipMemcpyHostToDevice, c.stream));
        GFR_HIP(hipMemcpyAsync(g.full.off, off.data(), 4ull * nf, hipMemcpyHostToDevice, c.stream));
        GFR_HIP(hipMemcpyAsync(g.full.row, row.data(), 4ull * nf, hipMemcpyHostToDevice, c.stream));
    }
    GFR_HIP(hipMemcpyAsync(g.full.part, part.data(), 4ull * (nch + 1), hipMemcpyHostToDevice, c.stream));
    GFR_HIP(hipMemcpyAsync(g.full_counts, counts, sizeof counts, hipMemcpyHostToDevice, c.stream));
    GFR_HIP(hipStreamSynchronize(c.stream));
    g.full_nf = nf;
    g.n_isolated = n - nf;
    g.bytes += g.full_mem.bytes;
}

// An output buffer the solvers can write on the device: the caller's own
// device buffer, or a staging buffer copied back to host memory afterwards.
struct OutBuf {
    void *user;
    void *dev;
    size_t bytes;
    bool staged;
    OutBuf(Ctx &c, void *p, size_t b) : user(p), dev(p), bytes(b), staged(false)
    {
        if (!p) fail(GFR_E_INVALID, "null output buffer");
        if (!is_device_ptr(p)) {
            if (c.stage.bytes < b) c.stage.alloc(b);
            dev = c.stage.p;
            staged = true;
        }
    }
    void finish(Ctx &c, hipStream_t s)
    {
        if (staged) copy_to_host(c.bounce, user, dev, bytes, s);
        GFR_HIP(hipStreamSynchronize(s));
    }
};

static hipStream_t pick_stream(Ctx &c, gfr_stream s) { return s ? (hipStream_t)s : c.stream; }

void deliver(Ctx &c, void *user, const void *dev, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (is_device_ptr(user)) GFR_HIP(hipMemcpyAsync(user, dev, bytes, hipMemcpyDeviceToDevice, s));
    else copy_to_host(c.bounce, user, dev, bytes, s);
    GFR_HIP(hipStreamSynchronize(s));
}

// seeds: host array of k distinct in-range vertices
static void check_seeds(const Graph &g, const int32_t *seeds, int32_t k, const char *who)
{
    if (k < 1 || !seeds) fail(GFR_E_INVALID, std::string(who) + ": need k >= 1 seeds");
    std::vector<uint8_t> seen((size_t)g.n, 0);
    for (int32_t i = 0; i < k; ++i) {
        if (seeds[i] < 0 || seeds[i] >= g.n) fail(GFR_E_INVALID, std::string(who) + ": seed out of range");
        if (seen[(size_t)seeds[i]]++) fail(GFR_E_INVALID, std::string(who) + ": duplicated seed");
    }
}

template <class F>
static gfr_status guard(gfr_ctx *ctx, F f)
{
    if (!ctx) return GFR_E_INVALID;
    Ctx &c = *(Ctx *)ctx;
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    try {
        c.err.clear();
        GFR_HIP(hipSetDevice(c.device));
        f(c);
        return GFR_OK;
    } catch (const Error &e) {
        c.err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        c.err = "host allocation failed";
        return GFR_E_OOM;
    } catch (const std::exception &e) {
        c.err = e.what();
        return GFR_E_DEVICE;
    }
}

static void timed_begin(Ctx &c, hipStream_t s)
{
    c.stats.clear();
    c.ktimer.reset();
    c.ktimer.on = c.opt.profile_kernels != 0;
    c.ktimer.advance_only = c.opt.profile_kernels == 2;
    GFR_HIP(hipEventRecord(c.ev0, s));
}

static void timed_end(Ctx &c, hipStream_t s)
{
    GFR_HIP(hipEventRecord(c.ev1, s));
    GFR_HIP(hipEventSynchronize(c.ev1));
    float ms = 0.f;
    GFR_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.stats.v["kernel_ms"] = ms;
    c.ktimer.collect(c.stats.v);
}

struct OptKey {
    const char *name;
    double lo, hi;
    bool per_graph;   // may be set per graph class by a tuning file
};

static const OptKey kOptKeys[] = {
    {"bfs.direction", 0, 2, true},       {"bfs.alpha", 1e-6, 1e9, true},
    {"bfs.beta", 1e-6, 1e9, true},       {"bfs.dedup", 0, 1, true},
    {"bfs.frontier", 0, 2, true},        {"sssp.frontier", 0, 2, true},
    {"sssp.delta", 0, 4.0e9, true},      {"advance.chunk", 256, 4096, true},
    {"sssp.delta_factor", 1e-3, 1e6, true}, {"batch.delta_factor", 0, 1e6, true},
    {"msbfs.alpha", 1e-6, 1e9, true},    {"batch.delta", 0, 4.0e9, true},
    {"batch.min_bfs", 1, 1e9, true},     {"batch.min_sssp", 1, 1e9, true},
    {"batch.pull_alpha", 0, 1e6, true},  {"batch.narrow", 0, 3, true},
    {"batch.blocks_per_cu", 0, 64, true}, {"graph.steps", 0, 1, false},
    {"batch.pair", 0, 1, true},          {"batch.pending", 0, 1, true},
    {"batch.sparse", 0, 64, true},
    {"advance.mapping", 0, 2, true},     {"advance.twc_threshold", 0, 2147483647.0, true},
    {"sssp.pull_alpha", 0, 1e6, true},
    {"bc.direction", 0, 2, true},
    {"bc.alpha", 1e-6, 1e9, true},       {"bc.beta", 1e-6, 1e9, true},
    {"twohop.direction", 0, 2, true},    {"twohop.alpha", 1e-6, 1e9, true},
    {"serve.budget_bytes", 0, 1e15, false}, {"serve.max_batch", 1, 64, false},
    {"profile.kernels", 0, 2, false}, {"serve.hipgraph", 0, 1, false},
};

static const OptKey &opt_key(const std::string &key)
{
    for (const auto &e : kOptKeys)
        if (key == e.name) return e;
    fail(GFR_E_INVALID, "unknown option '" + key + "'");
}

void option_set(Options &o, const std::string &key, double v)
{
    const OptKey &k = opt_key(key);
    if (!(v >= k.lo && v <= k.hi)) fail(GFR_E_INVALID, "option '" + key + "' out of range");
    if (key == "bfs.direction") o.bfs_direction = (int)v;
    else if (key == "bfs.alpha") o.bfs_alpha = v;
    else if (key == "bfs.beta") o.bfs_beta = v;
    else if (key == "bfs.dedup") o.bfs_dedup = (int)v;
    else if (key == "bfs.frontier") o.bfs_frontier = (int)v;
    else if (key == "sssp.frontier") o.sssp_frontier = (int)v;
    else if (key == "sssp.delta") o.sssp_delta = v;
    else if (key == "sssp.delta_factor") o.sssp_delta_factor = v;
    else if (key == "batch.delta_factor") o.batch_delta_factor = v;
    else if (key == "msbfs.alpha") o.msbfs_alpha = v;
    else if (key == "batch.delta") o.batch_delta = v;
    else if (key == "batch.min_bfs") o.batch_min_bfs = (int)v;
    else if (key == "batch.min_sssp") o.batch_min_sssp = (int)v;
    else if (key == "batch.pull_alpha") o.batch_pull_alpha = v;
    else if (key == "batch.blocks_per_cu") o.batch_blocks_per_cu = (int)v;
    else if (key == "graph.steps") o.step_graphs = (int)v;
    else if (key == "batch.pair") o.batch_pair = (int)v;
    else if (key == "batch.pending") o.batch_pending = (int)v;
    else if (key == "batch.sparse") o.batch_sparse = (int)v;
    else if (key == "advance.mapping") o.advance_mapping = (int)v;
    else if (key == "advance.twc_threshold") o.twc_threshold = (int)v;
    else if (key == "sssp.pull_alpha") o.sssp_pull_alpha = v;
    else if (key == "batch.narrow") o.batch_narrow = (int)v;
    else if (key == "bc.direction") o.bc_direction = (int)v;
    else if (key == "bc.alpha") o.bc_alpha = v;
    else if (key == "bc.beta") o.bc_beta = v;
    else if (key == "twohop.direction") o.twohop_direction = (int)v;
    else if (key == "twohop.alpha") o.twohop_alpha = v;
    else if (key == "serve.budget_bytes") o.serve_budget = v;
    else if (key == "serve.max_batch") o.serve_max_batch = (int)v;
    else if (key == "profile.kernels") o.profile_kernels = (int)v;
    else if (key == "serve.hipgraph") o.serve_graphs = (int)v;
    else if (key == "advance.chunk") {
        const int iv = (int)v;
        if (iv != 256 && iv != 512 && iv != 1024 && iv != 2048 && iv != 4096)
            fail(GFR_E_INVALID, "advance.chunk must be 256, 512, 1024, 2048 or 4096");
        o.advance_chunk = iv;
    }
}

static double option_get(const Options &o, const std::string &key)
{
    (void)opt_key(key);
    if (key == "bfs.direction") return o.bfs_direction;
    if (key == "bfs.alpha") return o.bfs_alpha;
    if (key == "bfs.beta") return o.bfs_beta;
    if (key == "bfs.dedup") return o.bfs_dedup;
    if (key == "bfs.frontier") return o.bfs_frontier;
    if (key == "sssp.frontier") return o.sssp_frontier;
    if (key == "sssp.delta") return o.sssp_delta;
    if (key == "sssp.delta_factor") return o.sssp_delta_factor;
    if (key == "batch.delta_factor") return o.batch_delta_factor;
    if (key == "advance.chunk") return o.advance_chunk;
    if (key == "msbfs.alpha") return o.msbfs_alpha;
    if (key == "batch.delta") return o.batch_delta;
    if (key == "batch.min_bfs") return o.batch_min_bfs;
    if (key == "batch.min_sssp") return o.batch_min_sssp;
    if (key == "batch.pull_alpha") return o.batch_pull_alpha;
    if (key == "batch.blocks_per_cu") return o.batch_blocks_per_cu;
    if (key == "graph.steps") return o.step_graphs;
    if (key == "batch.pair") return o.batch_pair;
    if (key == "batch.pending") return o.batch_pending;
    if (key == "batch.sparse") return o.batch_sparse;
    if (key == "advance.mapping") return o.advance_mapping;
    if (key == "advance.twc_threshold") return o.twc_threshold;
    if (key == "sssp.pull_alpha") return o.sssp_pull_alpha;
    if (key == "batch.narrow") return o.batch_narrow;
    if (key == "bc.direction") return o.bc_direction;
    if (key == "bc.alpha") return o.bc_alpha;
    if (key == "bc.beta") return o.bc_beta;
    if (key == "twohop.direction") return o.twohop_direction;
    if (key == "twohop.alpha") return o.twohop_alpha;
    if (key == "serve.budget_bytes") return o.serve_budget;
    if (key == "serve.max_batch") return o.serve_max_batch;
    if (key == "serve.hipgraph") return o.serve_graphs;
    return o.profile_kernels;
}

const char *const kClassNames[kNumGraphClasses] = {"scalefree", "mesh"};

int classify_graph(int32_t n, int64_t m, int32_t max_deg)
{
    const double mean = n > 0 ? (double)m / n : 0.0;
    return (double)max_deg >= 16.0 * (mean > 1.0 ? mean : 1.0) ? GRAPH_SCALEFREE : GRAPH_MESH;
}

// Parser for the tuning file: a JSON object whose members are numeric options
// (context-wide values) or objects named after a graph class holding
// per-graph numeric options for graphs of that class.  Validates every key
// and value; nothing is applied on error.
static void parse_tuning(const char *js, Tuning &t)
{
    std::string s(js);
    size_t i = 0;
    auto skip = [&]() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
    };
    auto key = [&]() {
        skip();
        if (i >= s.size() || s[i] != '"') fail(GFR_E_INVALID, "tuning_json: expected a key");
        size_t j = s.find('"', i + 1);
        if (j == std::string::npos) fail(GFR_E_INVALID, "tuning_json: unterminated key");
        std::string k = s.substr(i + 1, j - i - 1);
        i = j + 1;
        skip();
        if (i >= s.size() || s[i] != ':') fail(GFR_E_INVALID, "tuning_json: expected ':' after " + k);
        ++i;
        skip();
        return k;
    };
    auto number = [&](const std::string &k) {
        char *endp = nullptr;
        double v = strtod(s.c_str() + i, &endp);
        if (endp == s.c_str() + i) fail(GFR_E_INVALID, "tuning_json: expected a number for " + k);
        i = endp - s.c_str();
        return v;
    };
    // after a member: ',' then another member, or the closing brace
    auto next = [&]() {
        skip();
        if (i < s.size() && s[i] == ',') {
            ++i;
            return true;
        }
        if (i < s.size() && s[i] == '}') {
            ++i;
            return false;
        }
        fail(GFR_E_INVALID, "tuning_json: expected ',' or '}'");
    };
    auto open = [&]() {
        skip();
        if (i >= s.size() || s[i] != '{') fail(GFR_E_INVALID, "tuning_json: expected an object");
        ++i;
        skip();
        if (i < s.size() && s[i] == '}') {
            ++i;
            return false;
        }
        return true;
    };
    Options probe;
    for (bool more = open(); more; more = next()) {
        std::string k = key();
        int cls = -1;
        for (int c = 0; c < kNumGraphClasses; ++c)
            if (k == kClassNames[c]) cls = c;
        if (cls < 0) {
            double v = number(k);
            option_set(probe, k, v);
            t.global.push_back({k, v});
            continue;
        }
        for (bool inner = open(); inner; inner = next()) {
            std::string ck = key();
            double v = number(ck);
            if (!opt_key(ck).per_graph) fail(GFR_E_INVALID, "tuning_json: '" + ck + "' cannot be set per graph class");
            option_set(probe, ck, v);
            t.cls[cls].push_back({ck, v});
        }
    }
    skip();
    if (i != s.size()) fail(GFR_E_INVALID, "tuning_json: trailing characters");
}

Options effective_options(Ctx &c, const Graph &g)
{
    std::lock_guard<std::mutex> lo(c.opt_mu);
    Options o = c.base_opt;
    for (const auto &kv : c.tuning.cls[g.cls])
        if (!c.user_keys.count(kv.first)) option_set(o, kv.first, kv.second);
    return o;
}

OptScope::OptScope(Ctx &c, const Graph &g) : c(c), saved(c.opt)
{
    for (const auto &kv : c.tuning.cls[g.cls])
        if (!c.user_keys.count(kv.first)) option_set(c.opt, kv.first, kv.second);
}

OptScope::~OptScope() { c.opt = saved; }

}  // namespace gfr

using namespace gfr;

// Predecessor output of a single-source solve: written straight into a device
// buffer, or staged in the arena and copied out for host memory.
template <class Run>
static void with_pred(Ctx &c, Graph &g, int32_t *pred_out, hipStream_t s, Run run)
{
    if (!pred_out) return;
    int32_t *pd = pred_out;
    const bool dev = is_device_ptr(pred_out);
    if (!dev) {
        c.arena.reserve(al256(4ull * g.n));
        pd = c.arena.take<int32_t>(g.n);
    }
    run(pd);
    if (!dev) deliver(c, pred_out, pd, 4ull * g.n, s);
}

extern "C" {

gfr_status gfr_ctx_create(int32_t device, const char *tuning_json, gfr_ctx **out)
{
    if (!out) return GFR_E_INVALID;
    *out = nullptr;
    Tuning tuning;
    if (tuning_json) {
        try {
            parse_tuning(tuning_json, tuning);
        } catch (const Error &e) {
            return e.code;
        } catch (...) {
            return GFR_E_INVALID;
        }
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return GFR_E_DEVICE;
    }
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return GFR_E_OOM;
    gfr_status st = guard((gfr_ctx *)c, [&](Ctx &cc) {
        cc.device = device;
        GFR_HIP(hipSetDevice(device));
        hipDeviceProp_t p;
        GFR_HIP(hipGetDeviceProperties(&p, device));
        if (strncmp(p.gcnArchName, "gfx950", 6) != 0)
            fail(GFR_E_DEVICE, std::string("device is ") + p.gcnArchName + ", this library is built for gfx950");
        cc.num_cu = p.multiProcessorCount;
        // a blocking stream: work the caller queued earlier on the device's
        // null stream (PyTorch's default stream) finishes before ours starts
        GFR_HIP(hipStreamCreateWithFlags(&cc.stream, hipStreamDefault));
        cc.noalloc_scratch = noalloc_scratch(device);
        GFR_HIP(hipHostMalloc((void **)&cc.pinned, 4096, hipHostMallocDefault));
        GFR_HIP(hipEventCreate(&cc.ev0));
        GFR_HIP(hipEventCreate(&cc.ev1));
        cc.zero_word.alloc(256);
        GFR_HIP(hipMemsetAsync(cc.zero_word.p, 0, 256, cc.stream));
        GFR_HIP(hipStreamSynchronize(cc.stream));
        for (const auto &kv : tuning.global) option_set(cc.opt, kv.first, kv.second);
        std::lock_guard<std::mutex> lo(cc.opt_mu);
        cc.tuning = tuning;
        cc.base_opt = cc.opt;
    });
    if (st != GFR_OK) {
        gfr_ctx_destroy((gfr_ctx *)c);
        return st;
    }
    *out = (gfr_ctx *)c;
    return GFR_OK;
}

gfr_status gfr_ctx_destroy(gfr_ctx *ctx)
{
    if (!ctx) return GFR_OK;
    Ctx *c = (Ctx *)ctx;
    (void)hipSetDevice(c->device);
    serve_shutdown(*c);
    c->graphs.clear();
    c->step_graphs.clear();
    c->arena.mem.release();
    c->stage.release();
    c->zero_word.release();
    if (c->pinned) (void)hipHostFree(c->pinned);

    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return GFR_OK;
}

const char *gfr_last_error(const gfr_ctx *ctx)
{
    if (!ctx) return "null context";
    return ((const Ctx *)ctx)->err.c_str();
}

gfr_status gfr_set_option(gfr_ctx *ctx, const char *key, double value)
{
    return guard(ctx, [&](Ctx &c) {
        if (!key) fail(GFR_E_INVALID, "null key");
        option_set(c.opt, key, value);
        std::lock_guard<std::mutex> lo(c.opt_mu);
        option_set(c.base_opt, key, value);
        c.user_keys.insert(key);
    });
}

gfr_status gfr_get_option(gfr_ctx *ctx, const char *key, double *value)
{
    return guard(ctx, [&](Ctx &c) {
        if (!key || !value) fail(GFR_E_INVALID, "null argument");
        *value = option_get(c.opt, key);
    });
}

gfr_status gfr_get_stat(gfr_ctx *ctx, const char *key, double *value)
{
    return guard(ctx, [&](Ctx &c) {
        if (!key || !value) fail(GFR_E_INVALID, "null argument");
        if (serve_stat(c, key, value)) return;
        auto it = c.stats.v.find(key);
        if (it == c.stats.v.end()) fail(GFR_E_NOT_FOUND, std::string("no statistic '") + key + "'");
        *value = it->second;
    });
}

gfr_status gfr_validate_csr(int32_t n, int64_t m, const int32_t *R, const int32_t *C,
                            const uint32_t *W, uint32_t flags, char *msg, int32_t msg_cap)
{
    std::string why;
    try {
        why = check_csr(n, m, R, C, W, flags);
    } catch (...) {
        why = "validation failed";
    }
    if (msg && msg_cap > 0) {
        size_t k = std::min((size_t)msg_cap - 1, why.size());
        memcpy(msg, why.data(), k);
        msg[k] = 0;
    }
    return why.empty() ? GFR_OK : GFR_E_INVALID;
}

gfr_status gfr_graph_load_csr(gfr_ctx *ctx, int32_t n, int64_t m, const int32_t *R, const int32_t *C,
                              const uint32_t *W, uint32_t flags, gfr_graph *out)
{
    return guard(ctx, [&](Ctx &c) {
        if (!out) fail(GFR_E_INVALID, "null output handle");
        *out = 0;
        std::string why = check_csr(n, m, R, C, W, flags);
        if (!why.empty()) fail(GFR_E_INVALID, "graph_load_csr: " + why);
        auto g = std::make_unique<Graph>();
        g->n = n;
        g->m = m;
        g->R.alloc(4ull * (n + 1));
        g->C.alloc(4ull * std::max<int64_t>(m, 1));
        GFR_HIP(hipMemcpyAsync(g->R.p, R, 4ull * (n + 1), hipMemcpyHostToDevice, c.stream));
        if (m) GFR_HIP(hipMemcpyAsync(g->C.p, C, 4ull * m, hipMemcpyHostToDevice, c.stream));
        g->bytes = g->R.bytes + g->C.bytes;
        if (W) {
            g->W.alloc(4ull * std::max<int64_t>(m, 1));
            if (m) GFR_HIP(hipMemcpyAsync(g->W.p, W, 4ull * m, hipMemcpyHostToDevice, c.stream));
            g->weighted = true;
            g->bytes += g->W.bytes;
            double sw = 0;
            for (int64_t e = 0; e < m; ++e) sw += W[e];
            g->mean_w = m ? sw / (double)m : 1.0;
        }
        int32_t md = 0;
        for (int32_t i = 0; i < n; ++i) md = std::max(md, R[i + 1] - R[i]);
        g->max_deg = md;
        g->cls = classify_graph(n, m, md);
        build_full_queue(c, *g, R);
        GFR_HIP(hipStreamSynchronize(c.stream));
        const int64_t h = c.next_handle++;
        {
            std::lock_guard<std::mutex> lr(c.reg_mu);
            c.graphs[h] = std::move(g);
        }
        *out = h;
    });
}

gfr_status gfr_graph_free(gfr_ctx *ctx, gfr_graph g)
{
    return guard(ctx, [&](Ctx &c) {
        get_graph(c, g);
        GFR_HIP(hipStreamSynchronize(c.stream));
        if (!serve_release_graph(c, g))
            fail(GFR_E_NOT_READY, "graph_free: queries on this graph are queued or running");
    });
}

gfr_status gfr_graph_info(gfr_ctx *ctx, gfr_graph gh, int32_t *n, int64_t *m, uint64_t *bytes)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        if (n) *n = g.n;
        if (m) *m = g.m;
        if (bytes) *bytes = g.bytes;
    });
}

gfr_status gfr_bfs(gfr_ctx *ctx, gfr_graph gh, int32_t source, int32_t *depth_out, int32_t *pred_out,
                   gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (source < 0 || source >= g.n) fail(GFR_E_INVALID, "bfs: source out of range");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, depth_out, 4ull * g.n);
        timed_begin(c, s);
        run_bfs(c, g, source, (int32_t *)o.dev, s);
        with_pred(c, g, pred_out, s, [&](int32_t *pd) { run_bfs_pred(c, g, source, (const int32_t *)o.dev, pd, s); });
        timed_end(c, s);
        o.finish(c, s);
    });
}

gfr_status gfr_bfs_noalloc(gfr_ctx *ctx, gfr_graph gh, int32_t source, int32_t *depth_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (source < 0 || source >= g.n) fail(GFR_E_INVALID, "bfs_noalloc: source out of range");
        if (!depth_out || !is_device_ptr_on(depth_out, c.device))
            fail(GFR_E_INVALID, "bfs_noalloc: depth_out must be device memory of the context's device");
        if (!c.noalloc_scratch) fail(GFR_E_DEVICE, "bfs_noalloc: no scratch address for this device");
        hipStream_t s = pick_stream(c, stream);
        Arena ar(c.noalloc_scratch, GFR_NOALLOC_SCRATCH_BYTES);
        c.stats.clear();
        c.ktimer.reset();
        c.ktimer.on = false;   // per-launch timing would create events
        GFR_HIP(hipEventRecord(c.ev0, s));
        run_bfs(c, g, source, depth_out, s, ar);   // capacity is checked before any launch
        GFR_HIP(hipEventRecord(c.ev1, s));
        GFR_HIP(hipEventSynchronize(c.ev1));
        float ms = 0.f;
        GFR_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
        c.stats.v["kernel_ms"] = ms;
    });
}

gfr_status gfr_sssp(gfr_ctx *ctx, gfr_graph gh, int32_t source, uint32_t *dist_out, int32_t *pred_out,
                    gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (source < 0 || source >= g.n) fail(GFR_E_INVALID, "sssp: source out of range");
        if (!g.weighted) fail(GFR_E_INVALID, "sssp: graph was loaded without weights");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, dist_out, 4ull * g.n);
        timed_begin(c, s);
        run_sssp(c, g, source, (uint32_t *)o.dev, s);
        with_pred(c, g, pred_out, s,
                  [&](int32_t *pd) { run_sssp_pred(c, g, source, (const uint32_t *)o.dev, pd, s); });
        timed_end(c, s);
        o.finish(c, s);
    });
}

gfr_status gfr_bc(gfr_ctx *ctx, gfr_graph gh, const int32_t *sources, int32_t k, float *bc_out,
                  gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (k < 0 || (k > 0 && !sources)) fail(GFR_E_INVALID, "bc: bad source list");
        std::vector<int32_t> src(sources, sources + k);
        for (int32_t i = 0; i < k; ++i)
            if (src[i] < 0 || src[i] >= g.n) fail(GFR_E_INVALID, "bc: source out of range");
        std::vector<int32_t> sorted(src);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            fail(GFR_E_INVALID, "bc: duplicate source");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, bc_out, 4ull * g.n);
        timed_begin(c, s);
        run_bc(c, g, src.data(), k, (float *)o.dev, s);
        timed_end(c, s);
        o.finish(c, s);
    });
}

gfr_status gfr_cc(gfr_ctx *ctx, gfr_graph gh, int32_t *label_out, int32_t *num_components_out,
                  gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, label_out, 4ull * g.n);
        int32_t nc = 0;
        timed_begin(c, s);
        run_cc(c, g, (int32_t *)o.dev, &nc, s);
        timed_end(c, s);
        o.finish(c, s);
        if (num_components_out) *num_components_out = nc;
    });
}

gfr_status gfr_pagerank(gfr_ctx *ctx, gfr_graph gh, float damping, double l1_tol, int32_t max_iter,
                        float *rank_out, int32_t *iters_out, double *final_l1_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (!(damping > 0.f && damping < 1.f)) fail(GFR_E_INVALID, "pagerank: damping must be in (0,1)");
        if (max_iter < 1) fail(GFR_E_INVALID, "pagerank: max_iter must be >= 1");
        if (!(l1_tol >= 0.0)) fail(GFR_E_INVALID, "pagerank: l1_tol must be >= 0");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, rank_out, 4ull * g.n);
        int32_t it = 0;
        double l1 = 0.0;
        timed_begin(c, s);
        run_pagerank(c, g, damping, l1_tol, max_iter, (float *)o.dev, &it, &l1, s);
        timed_end(c, s);
        o.finish(c, s);
        if (iters_out) *iters_out = it;
        if (final_l1_out) *final_l1_out = l1;
    });
}

gfr_status gfr_pagerank_filtered(gfr_ctx *ctx, gfr_graph gh, double damping, double vertex_tol,
                                 int32_t max_iter, double *rank_out, uint8_t *active_out, int32_t *iters_out,
                                 double *final_l1_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (!(damping > 0.0 && damping < 1.0)) fail(GFR_E_INVALID, "pagerank_filtered: damping must be in (0,1)");
        if (max_iter < 1) fail(GFR_E_INVALID, "pagerank_filtered: max_iter must be >= 1");
        if (!(vertex_tol >= 0.0)) fail(GFR_E_INVALID, "pagerank_filtered: vertex_tol must be >= 0");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, rank_out, 8ull * g.n);
        int32_t it = 0;
        double l1 = 0.0;
        timed_begin(c, s);
        const uint8_t *act = run_pagerank_filtered(c, g, damping, vertex_tol, max_iter, (double *)o.dev, &it, &l1, s);
        timed_end(c, s);
        if (active_out) {
            if (is_device_ptr(active_out))
                GFR_HIP(hipMemcpyAsync(active_out, act, (size_t)g.n, hipMemcpyDeviceToDevice, s));
            else
                copy_to_host(c.bounce, active_out, act, (size_t)g.n, s);
        }
        o.finish(c, s);
        if (iters_out) *iters_out = it;
        if (final_l1_out) *final_l1_out = l1;
    });
}

static void need_device(const void *p, const char *what)
{
    if (p && !is_device_ptr(p)) fail(GFR_E_INVALID, std::string(what) + " must be device memory");
}

static gfr_status advance_call(gfr_ctx *ctx, gfr_graph gh, const int32_t *frontier, int32_t nf, bool edges,
                               int32_t *out_src, int32_t *out_edge, int32_t *out_dst, int64_t out_cap,
                               int64_t *count_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        const std::string who = edges ? "advance_edges" : "advance";
        Graph &g = get_graph(c, gh);
        if (nf < 0 || (nf > 0 && !frontier) || out_cap < 0 || !count_out) fail(GFR_E_INVALID, who + ": bad arguments");
        need_device(out_src, (who + ": out_src").c_str());
        need_device(out_edge, (who + ": out_edge").c_str());
        need_device(out_dst, (who + ": out_dst").c_str());
        hipStream_t s = pick_stream(c, stream);
        timed_begin(c, s);
        const int64_t total = run_advance(c, g, frontier, nf, edges, out_src, out_edge, out_dst, out_cap, s);
        timed_end(c, s);
        *count_out = total;
        if (total > out_cap) fail(GFR_E_CAPACITY, who + ": the edge frontier exceeds out_cap");
        if (total > INT32_MAX) fail(GFR_E_CAPACITY, who + ": more than 2^31 - 1 edges in one call");
    });
}

gfr_status gfr_advance(gfr_ctx *ctx, gfr_graph gh, const int32_t *frontier, int32_t nf, int32_t *out_src,
                       int32_t *out_edge, int32_t *out_dst, int64_t out_cap, int64_t *count_out, gfr_stream stream)
{
    return advance_call(ctx, gh, frontier, nf, false, out_src, out_edge, out_dst, out_cap, count_out, stream);
}

gfr_status gfr_advance_edges(gfr_ctx *ctx, gfr_graph gh, const int32_t *edges, int32_t ne, int32_t *out_src,
                             int32_t *out_edge, int32_t *out_dst, int64_t out_cap, int64_t *count_out,
                             gfr_stream stream)
{
    return advance_call(ctx, gh, edges, ne, true, out_src, out_edge, out_dst, out_cap, count_out, stream);
}

gfr_status gfr_filter(gfr_ctx *ctx, gfr_graph gh, const int32_t *items, int64_t count, const uint8_t *exclude,
                      int32_t *out, int64_t out_cap, int64_t *count_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        if (count < 0 || (count > 0 && !items) || out_cap < 0 || !count_out || (out_cap > 0 && !out))
            fail(GFR_E_INVALID, "filter: bad arguments");
        need_device(out, "filter: out");
        hipStream_t s = pick_stream(c, stream);
        timed_begin(c, s);
        const int64_t kept = run_filter(c, g, items, count, exclude, out, out_cap, s);
        timed_end(c, s);
        *count_out = kept;
        if (kept > out_cap) fail(GFR_E_CAPACITY, "filter: the result exceeds out_cap");
    });
}

gfr_status gfr_scan(gfr_ctx *ctx, const uint32_t *in, int64_t count, uint64_t *out, uint64_t *total_out,
                    gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        if (count < 0 || (count > 0 && (!in || !out))) fail(GFR_E_INVALID, "scan: bad arguments");
        need_device(out, "scan: out");
        hipStream_t s = pick_stream(c, stream);
        timed_begin(c, s);
        const uint64_t total = run_scan(c, in, count, (unsigned long long *)out, s);
        timed_end(c, s);
        if (total_out) *total_out = total;
    });
}

gfr_status gfr_split(gfr_ctx *ctx, gfr_graph gh, const int32_t *items, int64_t count, const uint32_t *dist,
                     uint32_t threshold, int32_t *near_out, int32_t *far_out, int64_t out_cap,
                     int64_t *near_count_out, int64_t *far_count_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        if (count < 0 || (count > 0 && (!items || !dist)) || out_cap < 0 || !near_count_out || !far_count_out ||
            (out_cap > 0 && (!near_out || !far_out)))
            fail(GFR_E_INVALID, "split: bad arguments");
        need_device(near_out, "split: near_out");
        need_device(far_out, "split: far_out");
        hipStream_t s = pick_stream(c, stream);
        timed_begin(c, s);
        int64_t nn = 0, nf = 0;
        run_split(c, g, items, count, dist, threshold, near_out, far_out, out_cap, &nn, &nf, s);
        timed_end(c, s);
        *near_count_out = nn;
        *far_count_out = nf;
        if (nn > out_cap || nf > out_cap) fail(GFR_E_CAPACITY, "split: a list exceeds out_cap");
    });
}

gfr_status gfr_two_hop(gfr_ctx *ctx, gfr_graph gh, const int32_t *seeds, int32_t k, uint64_t *count_out,
                       gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        check_seeds(g, seeds, k, "two_hop");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, count_out, 8ull * g.n);
        timed_begin(c, s);
        run_two_hop(c, g, seeds, k, (uint64_t *)o.dev, s);
        timed_end(c, s);
        o.finish(c, s);
    });
}

gfr_status gfr_ppr(gfr_ctx *ctx, gfr_graph gh, const int32_t *seeds, int32_t k, double damping, double l1_tol,
                   int32_t max_iter, double *rank_out, int32_t *iters_out, double *final_l1_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        check_seeds(g, seeds, k, "ppr");
        if (!(damping > 0.0 && damping < 1.0)) fail(GFR_E_INVALID, "ppr: damping must be in (0,1)");
        if (max_iter < 1) fail(GFR_E_INVALID, "ppr: max_iter must be >= 1");
        if (!(l1_tol >= 0.0)) fail(GFR_E_INVALID, "ppr: l1_tol must be >= 0");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, rank_out, 8ull * g.n);
        int32_t it = 0;
        double l1 = 0.0;
        timed_begin(c, s);
        run_ppr(c, g, seeds, k, damping, l1_tol, max_iter, (double *)o.dev, &it, &l1, s);
        timed_end(c, s);
        o.finish(c, s);
        if (iters_out) *iters_out = it;
        if (final_l1_out) *final_l1_out = l1;
    });
}

static gfr_status bipartite_rank(gfr_ctx *ctx, gfr_graph gh, int32_t n_left, int32_t iters, double *hub_out,
                                 double *auth_out, gfr_stream stream, bool walk)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        const char *who = walk ? "salsa" : "hits";
        if (n_left < 1 || n_left >= g.n) fail(GFR_E_INVALID, std::string(who) + ": need 0 < n_left < n");
        if (iters < 0) fail(GFR_E_INVALID, std::string(who) + ": iters must be >= 0");
        if (!hub_out || !auth_out) fail(GFR_E_INVALID, std::string(who) + ": null output buffer");
        hipStream_t s = pick_stream(c, stream);
        timed_begin(c, s);
        run_bipartite_rank(c, g, n_left, iters, walk, hub_out, auth_out, s);
        timed_end(c, s);
    });
}

gfr_status gfr_salsa(gfr_ctx *ctx, gfr_graph g, int32_t n_left, int32_t iters, double *hub_out, double *auth_out,
                     gfr_stream stream)
{
    return bipartite_rank(ctx, g, n_left, iters, hub_out, auth_out, stream, true);
}

gfr_status gfr_hits(gfr_ctx *ctx, gfr_graph g, int32_t n_left, int32_t iters, double *hub_out, double *auth_out,
                    gfr_stream stream)
{
    return bipartite_rank(ctx, g, n_left, iters, hub_out, auth_out, stream, false);
}

gfr_status gfr_bfs_batch(gfr_ctx *ctx, gfr_graph gh, const int32_t *sources, int32_t k,
                         int32_t *depth_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (k < 1 || !sources) fail(GFR_E_INVALID, "bfs_batch: need k >= 1 sources");
        for (int32_t i = 0; i < k; ++i)
            if (sources[i] < 0 || sources[i] >= g.n) fail(GFR_E_INVALID, "bfs_batch: source out of range");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, depth_out, 4ull * g.n * (size_t)k);
        timed_begin(c, s);
        run_bfs_batch(c, g, sources, k, (int32_t *)o.dev, s);
        timed_end(c, s);
        o.finish(c, s);
    });
}

gfr_status gfr_sssp_batch(gfr_ctx *ctx, gfr_graph gh, const int32_t *sources, int32_t k,
                          uint32_t *dist_out, gfr_stream stream)
{
    return guard(ctx, [&](Ctx &c) {
        Graph &g = get_graph(c, gh);
        OptScope os(c, g);
        if (k < 1 || !sources) fail(GFR_E_INVALID, "sssp_batch: need k >= 1 sources");
        if (!g.weighted) fail(GFR_E_INVALID, "sssp_batch: graph was loaded without weights");
        for (int32_t i = 0; i < k; ++i)
            if (sources[i] < 0 || sources[i] >= g.n) fail(GFR_E_INVALID, "sssp_batch: source out of range");
        hipStream_t s = pick_stream(c, stream);
        OutBuf o(c, dist_out, 4ull * g.n * (size_t)k);
        timed_begin(c, s);
        run_sssp_batch(c, g, sources, k, (uint32_t *)o.dev, s);
        timed_end(c, s);
        o.finish(c, s);
    });
}

}  // extern "C"
