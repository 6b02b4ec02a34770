// engine.h -- host-side internals of the frontier engine (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/gfr.h"
#include "device.h"

namespace gfr {

struct Error {
    gfr_status code;
    std::string msg;
};

[[noreturn]] void fail(gfr_status code, const std::string &msg);

#define GFR_HIP(x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            ::gfr::fail(e_ == hipErrorOutOfMemory ? GFR_E_OOM : GFR_E_DEVICE,               \
                        std::string(#x) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define GFR_LAUNCH_CHECK() GFR_HIP(hipGetLastError())

// Device allocation owned by RAII.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b)
    {
        release();
        if (b == 0) b = 256;
        GFR_HIP(hipMalloc(&p, b));
        bytes = b;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Scratch arena, carved per solve.  The context's arena grows (and only
// grows) by reallocating.  An arena over fixed device memory (second
// constructor) never allocates: a solve that needs more than it holds fails
// with GFR_E_CAPACITY before any device work is queued.
struct Arena {
    DevMem mem;
    char *fixed = nullptr;
    size_t fixed_bytes = 0;
    size_t used = 0;
    Arena() = default;
    Arena(void *p, size_t bytes) : fixed((char *)p), fixed_bytes(bytes) {}
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    char *base() const { return fixed ? fixed : (char *)mem.p; }
    size_t capacity() const { return fixed ? fixed_bytes : mem.bytes; }
    void reserve(size_t b)
    {
        used = 0;
        if (fixed) {
            if (b > fixed_bytes)
                fail(GFR_E_CAPACITY, "needs " + std::to_string(b) + " bytes of scratch; the fixed scratch holds " +
                                         std::to_string(fixed_bytes));
            return;
        }
        if (b > mem.bytes) mem.alloc(b + (b >> 3));
    }
    template <class T> T *take(size_t count)
    {
        size_t b = (count * sizeof(T) + 255) & ~(size_t)255;
        if (used + b > capacity()) fail(GFR_E_DEVICE, "internal: arena overflow");
        T *p = (T *)(base() + used);
        used += b;
        return p;
    }
};

static inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Graph classes for per-class tuning, chosen at load from the degree
// distribution (Sec. 7 suggests predicting parameters from it).
enum { GRAPH_SCALEFREE = 0, GRAPH_MESH = 1, kNumGraphClasses = 2 };
extern const char *const kClassNames[kNumGraphClasses];
// scale-free when the largest degree is at least 16 times the mean degree
int classify_graph(int32_t n, int64_t m, int32_t max_deg);

struct Graph {
    int32_t n = 0;
    int cls = GRAPH_MESH;
    int64_t m = 0;
    DevMem R, C, W;
    bool weighted = false;
    int32_t max_deg = 0;
    double mean_w = 0.0;
    uint64_t bytes = 0;
    // the whole vertex set as a frontier queue (non-isolated vertices in id
    // order, offsets = row offsets), chunked for the gather kernels
    FrontierQ full{};
    DevMem full_mem;
    uint32_t *full_counts = nullptr;   // device [nf, mf, 0, 0]
    int32_t full_nf = 0;
    int32_t n_isolated = 0;
    int32_t bip_checked_nl = -1;   // last side split verified for the bipartite rankings
    // hints for the speculative level loops (the size of the first batch of
    // launches), one per solver (a 64-source traversal takes more levels than
    // one source's); written by every solve on the graph, also from the
    // serving threads, hence atomic (relaxed: a stale hint only sizes a batch)
    std::atomic<int32_t> bfs_levels_hint{8};
    std::atomic<int32_t> sssp_iter_hint{16};
    std::atomic<int32_t> msbfs_levels_hint{8};
    std::atomic<int32_t> bsssp_iter_hint{16};
    int32_t levels_hint() const { return bfs_levels_hint.load(std::memory_order_relaxed); }
    int32_t iter_hint() const { return sssp_iter_hint.load(std::memory_order_relaxed); }
    // narrowest distance-row width (8, 16 or 32 bits) that no batched SSSP
    // on this graph has outgrown
    std::atomic<int> row_bits_min{8};
};

struct Options {
    int bfs_direction = 0;      // 0 auto, 1 push, 2 pull
    double bfs_alpha = 15.0;
    double bfs_beta = 18.0;
    int bfs_dedup = 0;          // 0 atomic, 1 idempotent
    int bfs_frontier = 0;       // 0 auto (mark bytes on mesh-class graphs), 1 queue, 2 mark bytes
    int sssp_frontier = 0;      // 0 auto (queue iterations), 1 queue, 2 mark bytes
    double sssp_pull_alpha = 0.0;   // single-source SSSP: pull sweep when the near queue's edges exceed m / alpha (0: never)
    double sssp_delta = 0.0;    // 0 -> sssp_delta_factor x mean edge weight
    double sssp_delta_factor = 2.0;
    int advance_chunk = 1024;
    int advance_mapping = 1;    // push work mapping (Sec. 4.4): 0 by frontier size, 1 edge chunks, 2 per-vertex groups
    int twc_threshold = 4096;   // mapping 0: per-vertex groups below this many frontier vertices
    double serve_budget = 32.0e9;
    int profile_kernels = 0;
    double msbfs_alpha = 4.0;   // batched BFS: pull when frontier edges > m / alpha
    double batch_delta = 0.0;   // batched SSSP bucket width; 0 -> batch_delta_factor
    double batch_delta_factor = 0.0;   // x mean edge weight; 0 -> one bucket (frontier order)
    double batch_pull_alpha = 0.0;     // batched SSSP: pull sweep when frontier edges > m / alpha (0: never)
    int batch_narrow = 0;       // batched SSSP narrow rows: 0 never, 1 auto, 2 from 16 bits, 3 from 8 bits
    int batch_blocks_per_cu = 64;  // batched SSSP relax grid: work-groups per CU, 0 = as many as are resident
    int batch_pair = 0;         // batched SSSP, 32-bit rows: relax two edges per row instruction
    int batch_pending = 1;      // batched SSSP: sources also relax queries improved earlier in the launch
    int batch_sparse = 8;       // batched SSSP: edge groups with at most this many queries per edge go lane = edge
    int step_graphs = 0;        // replay level steps from captured hipGraphs
    int serve_max_batch = 64;
    int serve_graphs = 1;       // serving sessions replay their rounds from captured hipGraphs
    int batch_min_bfs = 8;      // fewer sources than this: sequential single-source BFS
    int batch_min_sssp = 24;    // fewer queries than this: sequential single-source SSSP
    int bc_direction = 0;       // BC forward discovery: 0 auto, 1 push, 2 pull
    double bc_alpha = 15.0;     // push -> pull when level edges > unvisited edges / alpha (growing)
    double bc_beta = 18.0;      // pull -> push when level size < n / beta (shrinking)
    int twohop_direction = 0;   // 2-hop second advance: 0 auto, 1 push, 2 pull
    double twohop_alpha = 10.0; // auto: pull when the middle frontier's edges exceed m / alpha
};

// Options from a tuning file: context-wide values and per-graph-class values.
struct Tuning {
    std::vector<std::pair<std::string, double>> global;
    std::vector<std::pair<std::string, double>> cls[kNumGraphClasses];
};

void option_set(Options &o, const std::string &key, double v);

struct Stats {
    std::map<std::string, double> v;
    void clear() { v.clear(); }
};

struct Server;

// Two pinned chunks for copies into pageable host memory (see copy_to_host).
struct Bounce {
    char *buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    Bounce() = default;
    Bounce(const Bounce &) = delete;
    Bounce &operator=(const Bounce &) = delete;
    ~Bounce()
    {
        for (int i = 0; i < 2; ++i) {
            if (buf[i]) (void)hipHostFree(buf[i]);
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    }
};

// Copy `bytes` of device memory to host memory `dst` on stream s and wait for
// it.  Pinned destinations take one DMA; pageable ones go through the two
// pinned chunks of `b`, the DMA of one chunk overlapping the threaded host
// copy of the previous one.
void copy_to_host(Bounce &b, void *dst, const void *src, size_t bytes, hipStream_t s);

// Optional per-launch timing of named kernels with HIP events on the launch
// stream ("profile.kernels" option).  Results land in the context statistics
// as "t.<kernel>.ms" (summed device time) and "t.<kernel>.n" (launches).
// With advance_only, only the advance kernels (names holding "level",
// "relax" or "pull") are timed: each timed launch costs two event records.
struct KernelTimer {
    bool on = false;
    bool advance_only = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<const char *, std::pair<hipEvent_t, hipEvent_t>>> marks;
    size_t used = 0;
    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            GFR_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset()
    {
        used = 0;
        marks.clear();
    }
    static bool is_advance(const char *name)
    {
        return strstr(name, "level") || strstr(name, "relax") || strstr(name, "pull");
    }
    template <class F> void run(const char *name, hipStream_t s, F launch)
    {
        if (!on || (advance_only && !is_advance(name))) {
            launch();
            return;
        }
        hipEvent_t a = take(), b = take();
        GFR_HIP(hipEventRecord(a, s));
        launch();
        GFR_HIP(hipEventRecord(b, s));
        marks.push_back({name, {a, b}});
    }
    void collect(std::map<std::string, double> &out)
    {
        for (auto &m : marks) {
            GFR_HIP(hipEventSynchronize(m.second.second));
            float ms = 0.f;
            GFR_HIP(hipEventElapsedTime(&ms, m.second.first, m.second.second));
            out[std::string("t.") + m.first + ".ms"] += ms;
            out[std::string("t.") + m.first + ".n"] += 1.0;
        }
        reset();
    }
    ~KernelTimer()
    {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Captured level steps of the speculative level loop: a batch of k step
// launches is captured into a hipGraph the first time and replayed after.
// The key holds the bytes of every argument and the geometry of the step's
// launches, so a replay launches exactly what the direct launches would; the
// kernels read all state that changes from device memory.
struct StepGraphs {
    struct Entry {
        std::string key;
        int32_t k;
        hipGraphExec_t exec;
        uint64_t last;
    };
    std::vector<Entry> v;
    uint64_t tick = 0;
    static constexpr size_t kMax = 64;
    StepGraphs() = default;
    StepGraphs(const StepGraphs &) = delete;
    StepGraphs &operator=(const StepGraphs &) = delete;
    hipGraphExec_t find(const std::string &key, int32_t k)
    {
        for (auto &e : v)
            if (e.k == k && e.key == key) {
                e.last = ++tick;
                return e.exec;
            }
        return nullptr;
    }
    void put(const std::string &key, int32_t k, hipGraphExec_t exec)
    {
        if (v.size() >= kMax) {
            size_t old = 0;
            for (size_t i = 1; i < v.size(); ++i)
                if (v[i].last < v[old].last) old = i;
            (void)hipGraphExecDestroy(v[old].exec);
            v.erase(v.begin() + (long)old);
        }
        v.push_back({key, k, exec, ++tick});
    }
    void clear()
    {
        for (auto &e : v) (void)hipGraphExecDestroy(e.exec);
        v.clear();
    }
    ~StepGraphs() { clear(); }
};

// Key bytes of a step: append every launch argument struct (zero-filled
// before its fields were set, so padding compares equal) and the geometry.
struct StepKey {
    std::string k;
    explicit StepKey(const char *tag) : k(tag) { k.push_back('\0'); }
    template <class T> StepKey &add(const T &x)
    {
        k.append((const char *)&x, sizeof(T));
        return *this;
    }
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::recursive_mutex mu;      // serialises device work and most API calls
    std::mutex reg_mu;            // graph registry: held (with mu) to insert/erase, alone to look up
    std::mutex srv_mu;            // creation of the serving runtime
    std::string err;
    std::map<int64_t, std::unique_ptr<Graph>> graphs;
    int64_t next_handle = 1;
    Arena arena;
    void *noalloc_scratch = nullptr;   // this device's fixed scratch (gfr_bfs_noalloc)
    DevMem stage;                 // device staging for host output buffers
    DevMem zero_word;             // a device word that always holds 0
    uint32_t *pinned = nullptr;   // small pinned host buffer for control readbacks
    Options opt;                  // in effect; per-class values are applied by OptScope
    Tuning tuning;
    std::set<std::string> user_keys;   // options set by gfr_set_option (they beat the tuning file)
    Stats stats;
    Server *server = nullptr;     // owned; destroyed by serve_shutdown
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    KernelTimer ktimer;
    StepGraphs step_graphs;       // captured level steps, replayed by run_until_done
    Bounce bounce;                // for results written to pageable host memory
    // context-wide options as set (OptScope only changes `opt`), for the
    // serving thread, which holds opt_mu instead of mu to read them
    std::mutex opt_mu;
    Options base_opt;
};

// Options in effect for graph g (class values of the tuning file over the
// context-wide ones, except those set explicitly), read under c.opt_mu.
Options effective_options(Ctx &c, const Graph &g);

// While alive, c.opt holds the options for graph g: the tuning file's
// values for g's class over the context-wide ones, except for options the
// caller set explicitly.  The caller holds c.mu.
struct OptScope {
    Ctx &c;
    Options saved;
    OptScope(Ctx &c, const Graph &g);
    ~OptScope();
};

Graph &get_graph(Ctx &c, gfr_graph h);
bool is_device_ptr(const void *p);
int grid_blocks(const Ctx &c, int per_cu = 4);
// Work-groups of GFR_BLOCK threads for a grid-stride kernel: per_cu per CU,
// or (per_cu = 0) as many as are resident at once on every CU, so that no
// work-group of a statically divided grid starts after the others finish.
int resident_grid(const Ctx &c, const void *kernel, int per_cu);

// Solvers (outputs are device pointers on the context's device).
void run_bfs(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s);
// the same with its scratch carved from `ar` (the context's arena, or fixed memory)
void run_bfs(Ctx &c, Graph &g, int32_t src, int32_t *depth, hipStream_t s, Arena &ar);
void run_sssp(Ctx &c, Graph &g, int32_t src, uint32_t *dist, hipStream_t s);
// Predecessors from finished distances (device pointers): the first neighbour one step closer.
void run_bfs_pred(Ctx &c, Graph &g, int32_t src, const int32_t *depth, int32_t *pred, hipStream_t s);
void run_sssp_pred(Ctx &c, Graph &g, int32_t src, const uint32_t *dist, int32_t *pred, hipStream_t s);
// Bucket width factor x mean edge weight, clamped to [1, 1e9].
uint32_t sssp_auto_delta(const Graph &g, double factor);
void run_cc(Ctx &c, Graph &g, int32_t *label, int32_t *ncomp, hipStream_t s);
void run_pagerank(Ctx &c, Graph &g, float damping, double tol, int32_t max_iter, float *rank,
                  int32_t *iters, double *l1, hipStream_t s);
void run_ppr(Ctx &c, Graph &g, const int32_t *seeds, int32_t k, double damping, double tol, int32_t max_iter,
             double *rank, int32_t *iters, double *l1, hipStream_t s);
void run_two_hop(Ctx &c, Graph &g, const int32_t *seeds, int32_t k, uint64_t *count, hipStream_t s);
// SALSA (walk = true) or HITS; hub / auth are the caller's buffers (device or host)
void run_bipartite_rank(Ctx &c, Graph &g, int32_t nl, int32_t iters, bool walk, double *hub, double *auth,
                        hipStream_t s);
// The operators alone.  Outputs are device pointers.  Both return the output
// size; when it exceeds out_cap nothing is written.  With edges = true the
// frontier holds edge ids and is advanced from the edges' far ends.
int64_t run_advance(Ctx &c, Graph &g, const int32_t *frontier, int32_t nf, bool edges, int32_t *out_src,
                    int32_t *out_edge, int32_t *out_dst, int64_t out_cap, hipStream_t s);
int64_t run_filter(Ctx &c, Graph &g, const int32_t *items, int64_t count, const uint8_t *exclude, int32_t *out,
                   int64_t out_cap, hipStream_t s);
// Exclusive uint64 prefix sum of `in` (host or device) into device `out`; returns the total.
uint64_t run_scan(Ctx &c, const uint32_t *in, int64_t count, unsigned long long *out, hipStream_t s);
// Near/far split of `items` by dist[item] < threshold into device lists, input order kept; the
// counts are always set, and nothing is written when either exceeds out_cap.
void run_split(Ctx &c, Graph &g, const int32_t *items, int64_t count, const uint32_t *dist, uint32_t threshold,
               int32_t *near, int32_t *far, int64_t out_cap, int64_t *n_near, int64_t *n_far, hipStream_t s);
// Copy `bytes` of device data to a caller's buffer (device or host memory) and wait.
void deliver(Ctx &c, void *user, const void *dev, size_t bytes, hipStream_t s);
// Per-vertex convergence filtering; returns the final frontier membership
// (n bytes in the context's arena, valid until the next solver call).
const uint8_t *run_pagerank_filtered(Ctx &c, Graph &g, double damping, double vertex_tol, int32_t max_iter,
                                     double *rank, int32_t *iters, double *l1, hipStream_t s);
void run_bc(Ctx &c, Graph &g, const int32_t *sources, int32_t k, float *bc, hipStream_t s);
void run_bfs_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, int32_t *depth,
                   hipStream_t s);
void run_sssp_batch(Ctx &c, Graph &g, const int32_t *sources, int32_t k, uint32_t *dist,
                    hipStream_t s);

// Edges per chunk of the gather / for-each-edge kernels and of the full queue.
constexpr uint32_t GATHER_CH = 1024;

// Stops the serving runtime of a context (no-op if none).
// A traversal with 64 lanes (one query each) that queries join and leave
// at level boundaries: the continuous-batching unit of the serving runtime.
// All work is queued on the session's own stream; nothing blocks except
// copy_to_host.  Lane results live in rows of a [64][n] stage.
struct LaneSession {
    virtual ~LaneSession()
    {
        for (auto &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
    }
    // (re)start lanes: lanes[i] begins a query from sources[i] at the next step
    virtual void admit(const int32_t *lanes, const int32_t *sources, int32_t count) = 0;
    // lanes that left (their results were taken); they stop taking part
    virtual void release(unsigned long long lanes) = 0;
    // queue one level / relaxation round and the status read-back
    virtual void enqueue_step() = 0;
    // work to queue once before a round (outside any captured graph)
    virtual void pre_round() {}
    // k steps (k = 1, 2, 4 or 8), then `done` is recorded; with `graphs` the k
    // steps are captured into a hipGraph once and replayed from then on
    void round(int k, bool graphs);
    hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
    bool capture_failed = false;
    // after `done`: lanes that still have work, and whether the device flagged an error
    virtual unsigned long long active() const = 0;
    virtual gfr_status failed(std::string &msg) const = 0;
    // make the stage rows of `lanes` hold their results (queued)
    virtual void extract(unsigned long long lanes) = 0;
    const void *row(int lane) const { return (const char *)stage + (size_t)lane * 4 * n; }
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t bytes = 0;
    int32_t n = 0;
    void *stage = nullptr;
};
std::unique_ptr<LaneSession> make_bfs_session(Ctx &c, Graph &g, const Options &o);
std::unique_ptr<LaneSession> make_sssp_session(Ctx &c, Graph &g, const Options &o);
// device bytes of one session (state + stage) for a graph of n vertices and m edges
uint64_t bfs_session_bytes(int64_t n, int64_t m, int num_cu);
uint64_t sssp_session_bytes(int64_t n, int64_t m, int num_cu);

void serve_shutdown(Ctx &c);
// Remove graph gh from the registry unless served queries on it are queued or
// running (then false); idle serving sessions on it are dropped first.
bool serve_release_graph(Ctx &c, int64_t gh);
// Serving statistics ("serve.*" keys); false if the key is not a serving key.
bool serve_stat(Ctx &c, const std::string &key, double *value);

// Fill helpers.
void fill_u32(void *p, uint32_t value, size_t count, hipStream_t s);

// Spin on a device word until the speculative level loop reports completion.
// Launches `launch()` batches and reads *flag (device) back after each batch.
// With a step key (and option "graph.steps" on, per-launch timing off), each
// batch of k steps is replayed from a hipGraph captured the first time that
// key and k were seen; a capture that fails falls back to direct launches.
template <class LaunchFn>
int32_t run_until_done(Ctx &c, const uint32_t *flag_dev, uint32_t done_value, int32_t first_batch,
                       int64_t max_launches, hipStream_t s, LaunchFn launch, const StepKey *key = nullptr)
{
    int64_t launched = 0;
    int32_t batch = first_batch < 1 ? 1 : first_batch;
    const bool graphs = key && c.opt.step_graphs && !c.ktimer.on;
    for (;;) {
        hipGraphExec_t exec = graphs ? c.step_graphs.find(key->k, batch) : nullptr;
        if (graphs && !exec) {
            hipGraph_t gr = nullptr;
            bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                for (int32_t i = 0; i < batch; ++i) launch();
                ok = hipStreamEndCapture(s, &gr) == hipSuccess && gr;
            }
            if (ok) ok = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (gr) (void)hipGraphDestroy(gr);
            if (ok) {
                c.step_graphs.put(key->k, batch, exec);
            } else {
                (void)hipGetLastError();
                exec = nullptr;
            }
        }
        if (exec) {
            GFR_HIP(hipGraphLaunch(exec, s));
            c.stats.v["graph_launches"] += 1.0;
        } else {
            for (int32_t i = 0; i < batch; ++i) launch();
        }
        GFR_LAUNCH_CHECK();
        launched += batch;
        GFR_HIP(hipMemcpyAsync(c.pinned, flag_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        GFR_HIP(hipStreamSynchronize(s));
        if (*(volatile uint32_t *)c.pinned == done_value) break;
        if (launched > max_launches) fail(GFR_E_DEVICE, "iteration watchdog: solve did not converge");
        batch = batch < 128 ? batch * 2 : 256;
    }
    return (int32_t)launched;
}

}  // namespace gfr
