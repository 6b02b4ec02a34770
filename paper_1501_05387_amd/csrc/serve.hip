// serve.hip -- asynchronous query serving with continuous batching:
// submit / poll / cancel.
//
// A worker thread per context drives *sessions*: one 64-lane batched
// traversal per (graph, kind) with work (msbfs.hip / sssp_batch.hip), each on
// its own stream.  A session advances one level (BFS) or one relaxation round
// (SSSP) per step.  At every step boundary the worker
//   * retires the lanes whose traversal has ended: their results are copied
//     to the queries' own buffers and the tickets complete;
//   * admits queued queries of that graph and kind into free lanes (up to
//     `serve.max_batch` lanes busy); they start at the next step while the
//     other lanes continue where they are;
//   * launches the next step.
// Sessions of different graphs or kinds run on separate streams, so their
// steps overlap on the device.  A session for a new (graph, kind) is created
// when enough queries for it wait (the batch size from which one shared
// traversal beats sequential solves, "batch.min_bfs" / "batch.min_sssp") and
// its device footprint fits `serve.budget_bytes` beside the existing ones
// (idle sessions are dropped to make room).  Fewer waiting queries go to a
// pool of threads that solve them one by one with the single-source solvers,
// concurrently with the sessions (four threads, each with its own stream and
// scratch memory).  While no query waits for a session it runs
// several steps per round (up to 8) before it is looked at again; the steps
// of a round are captured into a hipGraph once per session and replayed
// ("serve.hipgraph").
// With `serve.max_batch` = 1 every query takes the single-source path (the
// unbatched reference).
//
// Locks, always taken in this order: c.mu (device work of API calls) ->
// sv->sess_mu (the session list; the worker holds it while it touches
// sessions and never waits for c.mu under it) -> sv->mu (queue and tickets).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace gfr {

using Clock = std::chrono::steady_clock;

struct Ticket {
    gfr_query q;
    gfr_status status = GFR_OK;
    Clock::time_point t_submit, t_done;
    int state = 0;   // 0 queued, 1 running, 2 done
};

struct SessionEntry {
    std::unique_ptr<LaneSession> s;
    int64_t graph = 0;
    int32_t kind = 0;
    gfr_ticket lane[64] = {};
    unsigned long long busy = 0;
    bool in_flight = false;
    int round = 1;   // steps per round while no query waits for this session
    Clock::time_point last_used;
};

struct Server {
    Ctx *ctx = nullptr;
    std::thread worker;
    std::mutex mu;                 // queue, tickets, statistics
    std::condition_variable cv_work, cv_done;
    std::deque<gfr_ticket> queue;
    std::unordered_map<gfr_ticket, Ticket> tickets;
    std::deque<gfr_ticket> finished;
    std::deque<gfr_ticket> singles;   // for the single-source threads
    std::condition_variable cv_single;
    std::vector<std::thread> single_workers;
    int singles_running = 0;
    bool stop = false;
    gfr_ticket next = 1;
    std::mutex sess_mu;            // sessions (and their device memory)
    std::vector<std::unique_ptr<SessionEntry>> sessions;
    // results copied to device outputs, completed when their event has fired
    // (worker only, under sess_mu)
    struct PendingDone {
        hipEvent_t ev;
        std::vector<gfr_ticket> tickets;
    };
    std::vector<PendingDone> pending;
    std::vector<hipEvent_t> ev_pool;
    Bounce bounce;                 // host copies of the worker
    // statistics
    std::vector<double> latency_ms;
    uint64_t steps = 0, lane_steps = 0;
    uint64_t joined = 0;           // queries that joined a session with other lanes running
};

void LaneSession::round(int k, bool graphs)
{
    pre_round();
    const int idx = k >= 8 ? 3 : k >= 4 ? 2 : k >= 2 ? 1 : 0;
    k = 1 << idx;
    if (graphs && !capture_failed && !exec[idx]) {
        // capture the k steps once; kernel arguments never change, all state
        // lives in the session's device memory
        hipGraph_t gr = nullptr;
        bool ok = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (int i = 0; i < k; ++i) enqueue_step();
            ok = hipStreamEndCapture(stream, &gr) == hipSuccess && gr;
        }
        if (ok) ok = hipGraphInstantiate(&exec[idx], gr, nullptr, nullptr, 0) == hipSuccess;
        if (gr) (void)hipGraphDestroy(gr);
        if (!ok) {
            (void)hipGetLastError();
            exec[idx] = nullptr;
            capture_failed = true;
        }
    }
    if (graphs && exec[idx]) {
        GFR_HIP(hipGraphLaunch(exec[idx], stream));
    } else {
        for (int i = 0; i < k; ++i) enqueue_step();
    }
    GFR_HIP(hipEventRecord(done, stream));
}

static uint64_t session_bytes(const Ctx &c, const Graph &g, int32_t kind)
{
    return kind == GFR_Q_BFS ? bfs_session_bytes(g.n, g.m, c.num_cu) : sssp_session_bytes(g.n, g.m, c.num_cu);
}

// Under sv->mu.
static void complete_locked(Server *sv, gfr_ticket t, gfr_status st)
{
    Ticket &tk = sv->tickets[t];
    tk.state = 2;
    tk.status = st;
    tk.t_done = Clock::now();
    sv->latency_ms.push_back(std::chrono::duration<double, std::milli>(tk.t_done - tk.t_submit).count());
    sv->finished.push_back(t);
}

static gfr_query query_of(Server *sv, gfr_ticket t)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv->tickets[t].q;
}

// Copy finished lanes' results out, complete their tickets, free the lanes.
// When every output is device memory the copies are only queued: the lanes
// are free at once (anything later on the session's stream runs after the
// copies) and the tickets complete when the copies' event has fired, so the
// worker never waits for a session here.  Host outputs are copied through
// the bounce buffers and waited for.
static void retire(Server *sv, SessionEntry &e, unsigned long long lanes, gfr_status st)
{
    if (!lanes) return;
    LaneSession &s = *e.s;
    const size_t row = 4ull * (size_t)s.n;
    if (st == GFR_OK) {
        try {
            bool all_dev = true;
            for (unsigned long long m = lanes; m; m &= m - 1)
                all_dev &= query_of(sv, e.lane[__builtin_ctzll(m)]).out_on_device != 0;
            s.extract(lanes);
            for (unsigned long long m = lanes; m; m &= m - 1) {
                const int q = __builtin_ctzll(m);
                const gfr_query qq = query_of(sv, e.lane[q]);
                if (qq.out_on_device)
                    GFR_HIP(hipMemcpyAsync(qq.out, s.row(q), row, hipMemcpyDeviceToDevice, s.stream));
                else
                    copy_to_host(sv->bounce, qq.out, s.row(q), row, s.stream);
            }
            if (all_dev) {
                hipEvent_t ev = nullptr;
                if (!sv->ev_pool.empty()) {
                    ev = sv->ev_pool.back();
                    sv->ev_pool.pop_back();
                } else {
                    GFR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                }
                GFR_HIP(hipEventRecord(ev, s.stream));
                Server::PendingDone p{ev, {}};
                for (unsigned long long m = lanes; m; m &= m - 1) {
                    const int q = __builtin_ctzll(m);
                    p.tickets.push_back(e.lane[q]);
                    e.lane[q] = 0;
                }
                sv->pending.push_back(std::move(p));
                e.busy &= ~lanes;
                s.release(lanes);
                return;
            }
            GFR_HIP(hipStreamSynchronize(s.stream));
        } catch (const Error &err) {
            st = err.code;
        }
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (unsigned long long m = lanes; m; m &= m - 1) {
            const int q = __builtin_ctzll(m);
            complete_locked(sv, e.lane[q], st);
            e.lane[q] = 0;
        }
    }
    e.busy &= ~lanes;
    s.release(lanes);
    sv->cv_done.notify_all();
}

// Complete the tickets whose result copies have finished (under sess_mu).
static bool complete_pending(Server *sv)
{
    bool any = false;
    for (size_t i = 0; i < sv->pending.size();) {
        Server::PendingDone &p = sv->pending[i];
        const hipError_t r = hipEventQuery(p.ev);
        if (r == hipErrorNotReady) {
            ++i;
            continue;
        }
        gfr_status st = GFR_OK;
        if (r != hipSuccess) {
            (void)hipGetLastError();
            st = GFR_E_DEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (gfr_ticket t : p.tickets) complete_locked(sv, t, st);
        }
        sv->ev_pool.push_back(p.ev);
        sv->pending.erase(sv->pending.begin() + (long)i);
        any = true;
    }
    if (any) sv->cv_done.notify_all();
    return any;
}

// Private device state of a single-source thread: its own stream, scratch
// arena and staging, so that several queries are solved at once beside the
// sessions and the caller's own calls.
struct SingleCtx {
    Ctx c;
    DevMem stage;
    Bounce bounce;
    explicit SingleCtx(const Ctx &main)
    {
        c.device = main.device;
        c.num_cu = main.num_cu;
        GFR_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        GFR_HIP(hipHostMalloc((void **)&c.pinned, 4096, hipHostMallocDefault));
    }
    ~SingleCtx()
    {
        if (c.stream) (void)hipStreamSynchronize(c.stream);
        if (c.pinned) (void)hipHostFree(c.pinned);
        if (c.stream) (void)hipStreamDestroy(c.stream);
    }
};

// One query through the single-source solver.
static void run_one(Server *sv, SingleCtx &sc, gfr_ticket t)
{
    Ctx &c = *sv->ctx;
    const gfr_query q = query_of(sv, t);
    gfr_status st = GFR_OK;
    try {
        Graph *g = nullptr;
        {
            std::lock_guard<std::mutex> lr(c.reg_mu);
            auto git = c.graphs.find(q.graph);
            if (git == c.graphs.end()) fail(GFR_E_NOT_FOUND, "graph is gone");
            g = git->second.get();   // kept alive: the ticket is running
        }
        sc.c.opt = effective_options(c, *g);
        sc.c.stats.clear();
        sc.c.ktimer.on = false;
        const size_t row = 4ull * g->n;
        if (sc.stage.bytes < row) sc.stage.alloc(row);
        hipStream_t s = sc.c.stream;
        if (q.kind == GFR_Q_BFS) run_bfs(sc.c, *g, q.source, sc.stage.as<int32_t>(), s);
        else run_sssp(sc.c, *g, q.source, sc.stage.as<uint32_t>(), s);
        if (q.out_on_device) GFR_HIP(hipMemcpyAsync(q.out, sc.stage.p, row, hipMemcpyDeviceToDevice, s));
        else copy_to_host(sc.bounce, q.out, sc.stage.p, row, s);
        GFR_HIP(hipStreamSynchronize(s));
    } catch (const Error &e) {
        st = e.code;
    } catch (...) {
        st = GFR_E_DEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        complete_locked(sv, t, st);
        sv->steps += 1;
        sv->lane_steps += 1;
    }
    sv->cv_done.notify_all();
}

// Thread `id` of the single-source pool; with serve.max_batch = 1 only
// thread 0 takes queries, so they run strictly one at a time.
constexpr int kSingleThreads = 4;

static void single_loop(Server *sv, int id)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_ptr<SingleCtx> sc;
    for (;;) {
        gfr_ticket t = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_single.wait(lk, [&] {
                if (sv->stop) return true;
                if (sv->singles.empty()) return false;
                if (id == 0) return true;
                std::lock_guard<std::mutex> lo(sv->ctx->opt_mu);
                return sv->ctx->base_opt.serve_max_batch > 1;
            });
            if (sv->stop) return;
            t = sv->singles.front();
            sv->singles.pop_front();
            sv->singles_running += 1;
        }
        try {
            if (!sc) sc.reset(new SingleCtx(*sv->ctx));
            run_one(sv, *sc, t);
        } catch (const Error &e) {
            std::lock_guard<std::mutex> lk(sv->mu);
            complete_locked(sv, t, e.code);
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->singles_running -= 1;
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_one();
    }
}

struct Admit {
    SessionEntry *e;
    int32_t lane, source;
};

static void drop_dead_sessions(Server *sv)
{
    sv->sessions.erase(std::remove_if(sv->sessions.begin(), sv->sessions.end(),
                                      [](const std::unique_ptr<SessionEntry> &e) { return !e->s; }),
                       sv->sessions.end());
}

static void worker_loop(Server *sv)
{
    Ctx &c = *sv->ctx;
    (void)hipSetDevice(c.device);
    for (;;) {
        int max_batch;
        double budget;
        bool use_graphs;
        {
            std::lock_guard<std::mutex> lo(c.opt_mu);
            max_batch = std::max(1, std::min(64, c.base_opt.serve_max_batch));
            budget = c.base_opt.serve_budget;
            use_graphs = c.base_opt.serve_graphs != 0;
        }
        // unbatched reference: every query through the single-source thread
        if (max_batch == 1) {
            bool idle;
            {
                std::lock_guard<std::mutex> ls(sv->sess_mu);
                idle = std::none_of(sv->sessions.begin(), sv->sessions.end(),
                                    [](const std::unique_ptr<SessionEntry> &e) { return e->busy != 0; });
                if (idle) sv->sessions.clear();
            }
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->stop) return;
            if (idle) {   // once the sessions have drained
                while (!sv->queue.empty()) {
                    sv->tickets[sv->queue.front()].state = 1;
                    sv->singles.push_back(sv->queue.front());
                    sv->queue.pop_front();
                }
                sv->cv_single.notify_one();
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(2), [&] { return sv->stop || !sv->queue.empty(); });
                if (sv->stop) return;
                continue;
            }
        }
        bool in_flight = false, progress = false;
        {
            std::unique_lock<std::mutex> ls(sv->sess_mu);
            progress |= complete_pending(sv);
            // 1. steps that ended: retire the lanes that finished
            for (auto &ep : sv->sessions) {
                SessionEntry &e = *ep;
                if (!e.in_flight) continue;
                const hipError_t r = hipEventQuery(e.s->done);
                if (r == hipErrorNotReady) continue;
                e.in_flight = false;
                progress = true;
                std::string msg;
                gfr_status st = GFR_E_DEVICE;
                if (r == hipSuccess) st = e.s->failed(msg);
                else (void)hipGetLastError();
                retire(sv, e, st == GFR_OK ? (e.busy & ~e.s->active()) : e.busy, st);
                if (st != GFR_OK) e.s.reset();   // rebuilt on demand
                e.last_used = Clock::now();
            }
            drop_dead_sessions(sv);
            // 2. admissions into sessions at a step boundary, in arrival order
            std::vector<Admit> plan;
            std::vector<std::pair<int64_t, int32_t>> wanted;   // (graph, kind) without a session
            std::vector<std::pair<int64_t, int32_t>> waiting;  // keys with queries still queued
            // batch-size crossovers of the graphs in the queue (their class options)
            std::unordered_map<int64_t, std::pair<int, int>> min_batch;
            {
                std::vector<int64_t> gs;
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    for (gfr_ticket id : sv->queue) {
                        const int64_t gh = sv->tickets[id].q.graph;
                        if (std::find(gs.begin(), gs.end(), gh) == gs.end()) gs.push_back(gh);
                    }
                }
                for (int64_t gh : gs) {
                    Graph *g = nullptr;
                    {
                        std::lock_guard<std::mutex> lr(c.reg_mu);
                        auto git = c.graphs.find(gh);
                        if (git != c.graphs.end()) g = git->second.get();
                    }
                    if (!g) continue;
                    const Options o = effective_options(c, *g);
                    min_batch[gh] = {o.batch_min_bfs, o.batch_min_sssp};
                }
            }
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (sv->stop) return;
                std::vector<std::pair<std::pair<int64_t, int32_t>, int>> count;
                for (gfr_ticket id : sv->queue) {
                    const std::pair<int64_t, int32_t> key(sv->tickets[id].q.graph, sv->tickets[id].q.kind);
                    auto f = std::find_if(count.begin(), count.end(), [&](const auto &x) { return x.first == key; });
                    if (f == count.end()) count.push_back({key, 1});
                    else f->second += 1;
                }
                for (auto it = sv->queue.begin(); it != sv->queue.end();) {
                    Ticket &t = sv->tickets[*it];
                    const std::pair<int64_t, int32_t> key(t.q.graph, t.q.kind);
                    SessionEntry *e = nullptr;
                    for (auto &ep : sv->sessions)
                        if (ep->graph == t.q.graph && ep->kind == t.q.kind) e = ep.get();
                    if (!e || !e->busy) {
                        // no running session: batch only if enough queries wait,
                        // else solve singly when the single-source thread is free
                        const auto mb = min_batch.find(t.q.graph);
                        const int need = mb == min_batch.end()
                                             ? 1
                                             : std::min(max_batch, t.q.kind == GFR_Q_BFS ? mb->second.first
                                                                                         : mb->second.second);
                        const int have = std::find_if(count.begin(), count.end(),
                                                      [&](const auto &x) { return x.first == key; })->second;
                        if (have < need) {
                            if (sv->singles_running + (int)sv->singles.size() < kSingleThreads) {
                                t.state = 1;
                                sv->singles.push_back(*it);
                                sv->cv_single.notify_one();
                                it = sv->queue.erase(it);
                            } else {
                                ++it;
                            }
                            continue;
                        }
                        if (!e) {
                            if (std::find(wanted.begin(), wanted.end(), key) == wanted.end()) wanted.push_back(key);
                            ++it;
                            continue;
                        }
                    }
                    if (e->in_flight || __builtin_popcountll(e->busy) >= max_batch) {
                        if (std::find(waiting.begin(), waiting.end(), key) == waiting.end()) waiting.push_back(key);
                        ++it;
                        continue;
                    }
                    const int lane = __builtin_ctzll(~e->busy);
                    if (e->busy) sv->joined += 1;
                    e->busy |= 1ull << lane;
                    e->lane[lane] = *it;
                    t.state = 1;
                    plan.push_back({e, lane, t.q.source});
                    it = sv->queue.erase(it);
                }
            }
            // 3. a lowered budget releases idle sessions beyond it; new
            //    sessions open where the budget allows (idle ones make room),
            //    and their queries are admitted on the next pass
            {
                uint64_t used = 0;
                for (auto &ep : sv->sessions) used += ep->s->bytes;
                while ((double)used > budget) {
                    auto victim = sv->sessions.end();
                    for (auto it = sv->sessions.begin(); it != sv->sessions.end(); ++it)
                        if (!(*it)->busy && !(*it)->in_flight &&
                            (victim == sv->sessions.end() || (*it)->last_used < (*victim)->last_used))
                            victim = it;
                    if (victim == sv->sessions.end()) break;
                    used -= (*victim)->s->bytes;
                    sv->sessions.erase(victim);
                }
            }
            if (!wanted.empty()) {
                uint64_t used = 0;
                for (auto &ep : sv->sessions) used += ep->s->bytes;
                for (const auto &key : wanted) {
                    Graph *g = nullptr;
                    {
                        std::lock_guard<std::mutex> lr(c.reg_mu);
                        auto git = c.graphs.find(key.first);
                        if (git != c.graphs.end()) g = git->second.get();
                    }
                    if (!g) continue;   // its queries fail below
                    const uint64_t need = session_bytes(c, *g, key.second);
                    while ((double)(used + need) > budget) {
                        auto victim = sv->sessions.end();
                        for (auto it = sv->sessions.begin(); it != sv->sessions.end(); ++it)
                            if (!(*it)->busy && !(*it)->in_flight &&
                                (victim == sv->sessions.end() || (*it)->last_used < (*victim)->last_used))
                                victim = it;
                        if (victim == sv->sessions.end()) break;
                        used -= (*victim)->s->bytes;
                        sv->sessions.erase(victim);
                    }
                    if ((double)(used + need) > budget) continue;   // waits for room
                    std::unique_ptr<SessionEntry> e(new SessionEntry());
                    e->graph = key.first;
                    e->kind = key.second;
                    e->last_used = Clock::now();
                    try {
                        const Options o = effective_options(c, *g);
                        e->s = key.second == GFR_Q_BFS ? make_bfs_session(c, *g, o) : make_sssp_session(c, *g, o);
                    } catch (const Error &) {
                        continue;   // device memory short: its queries wait
                    }
                    used += e->s->bytes;
                    sv->sessions.push_back(std::move(e));
                    progress = true;
                }
            }
            // queries on graphs that no longer exist fail
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                std::lock_guard<std::mutex> lr(c.reg_mu);
                for (auto it = sv->queue.begin(); it != sv->queue.end();) {
                    if (!c.graphs.count(sv->tickets[*it].q.graph)) {
                        complete_locked(sv, *it, GFR_E_NOT_FOUND);
                        it = sv->queue.erase(it);
                        progress = true;
                    } else {
                        ++it;
                    }
                }
            }
            // 4. start the admitted lanes and launch the next steps
            for (auto &ep : sv->sessions) {
                SessionEntry &e = *ep;
                std::vector<int32_t> lanes, srcs;
                for (const Admit &a : plan)
                    if (a.e == &e) {
                        lanes.push_back(a.lane);
                        srcs.push_back(a.source);
                    }
                try {
                    if (!lanes.empty()) e.s->admit(lanes.data(), srcs.data(), (int32_t)lanes.size());
                    if (e.busy && !e.in_flight) {
                        // several steps per round unless queries wait to join
                        const bool wait = std::find(waiting.begin(), waiting.end(),
                                                    std::make_pair(e.graph, e.kind)) != waiting.end();
                        e.round = wait ? 1 : std::min(8, e.round * 2);
                        e.s->round(e.round, use_graphs);
                        e.in_flight = true;
                        std::lock_guard<std::mutex> lk(sv->mu);
                        sv->steps += (uint64_t)e.round;
                        sv->lane_steps += (uint64_t)e.round * (uint64_t)__builtin_popcountll(e.busy);
                    }
                } catch (const Error &err) {
                    retire(sv, e, e.busy, err.code);
                    e.s.reset();
                }
                if (e.s && e.in_flight) in_flight = true;
            }
            drop_dead_sessions(sv);
            if (!sv->pending.empty()) in_flight = true;
        }
        sv->cv_done.notify_all();
        if (in_flight) {
            if (!progress) std::this_thread::yield();
        } else {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait_for(lk, std::chrono::milliseconds(2), [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->stop) return;
        }
    }
}

void serve_shutdown(Ctx &c)
{
    Server *sv = c.server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_single.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (auto &th : sv->single_workers)
        if (th.joinable()) th.join();
    for (auto &p : sv->pending) {
        (void)hipEventSynchronize(p.ev);
        (void)hipEventDestroy(p.ev);
    }
    for (hipEvent_t ev : sv->ev_pool) (void)hipEventDestroy(ev);
    delete sv;   // session destructors wait for their streams
    c.server = nullptr;
}

// The context's server, created on first use (under its own mutex, so that
// submit / poll never wait for device work).
static Server &server_of(Ctx &c)
{
    std::lock_guard<std::mutex> ls(c.srv_mu);
    if (!c.server) {
        Server *sv = new Server();
        sv->ctx = &c;
        c.server = sv;
        sv->worker = std::thread(worker_loop, sv);
        for (int i = 0; i < kSingleThreads; ++i) sv->single_workers.emplace_back(single_loop, sv, i);
    }
    return *c.server;
}

bool serve_release_graph(Ctx &c, int64_t gh)
{
    Server *sv;
    {
        std::lock_guard<std::mutex> ls(c.srv_mu);
        sv = c.server;
    }
    auto erase = [&]() {
        std::lock_guard<std::mutex> lr(c.reg_mu);
        c.graphs.erase(gh);
    };
    if (!sv) {
        erase();
        return true;
    }
    // under the session lock, so that no session is created for the graph
    // between the check and the erase (sessions are only made for queued
    // queries, after a registry lookup)
    std::lock_guard<std::mutex> ls(sv->sess_mu);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (const auto &kv : sv->tickets)
            if (kv.second.state < 2 && kv.second.q.graph == gh) return false;
    }
    // no query left on the graph: its sessions are idle
    sv->sessions.erase(std::remove_if(sv->sessions.begin(), sv->sessions.end(),
                                      [&](const std::unique_ptr<SessionEntry> &e) { return e->graph == gh; }),
                       sv->sessions.end());
    erase();
    return true;
}

// percentile of a copy of v (nearest rank)
static double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t i = (size_t)std::ceil(p / 100.0 * (double)v.size());
    if (i > 0) --i;
    return v[std::min(i, v.size() - 1)];
}

bool serve_stat(Ctx &c, const std::string &key, double *value)
{
    if (key.rfind("serve.", 0) != 0) return false;
    Server &sv = server_of(c);
    if (key == "serve.sessions" || key == "serve.session_bytes") {
        std::lock_guard<std::mutex> ls(sv.sess_mu);
        double x = 0;
        for (auto &e : sv.sessions) x += key == "serve.sessions" ? 1.0 : (double)e->s->bytes;
        *value = x;
        return true;
    }
    std::lock_guard<std::mutex> lk(sv.mu);
    if (key == "serve.completed") *value = (double)sv.latency_ms.size();
    else if (key == "serve.batches") *value = (double)sv.steps;
    else if (key == "serve.mean_batch") *value = sv.steps ? (double)sv.lane_steps / sv.steps : 0.0;
    else if (key == "serve.p50_ms") *value = percentile(sv.latency_ms, 50);
    else if (key == "serve.p99_ms") *value = percentile(sv.latency_ms, 99);
    else if (key == "serve.queued") *value = (double)sv.queue.size();
    else if (key == "serve.joined") *value = (double)sv.joined;
    else if (key == "serve.reset") {
        sv.latency_ms.clear();
        sv.steps = sv.lane_steps = sv.joined = 0;
        *value = 0.0;
    } else {
        fail(GFR_E_NOT_FOUND, "no statistic '" + key + "'");
    }
    return true;
}

}  // namespace gfr

using namespace gfr;

extern "C" {

gfr_status gfr_submit_queries(gfr_ctx *ctx, const gfr_query *queries, int32_t count, gfr_ticket *tickets_out)
{
    if (!ctx) return GFR_E_INVALID;
    Ctx &c = *(Ctx *)ctx;
    std::vector<Ticket> staged;
    if (count < 0 || (count > 0 && (!queries || !tickets_out))) return GFR_E_INVALID;
    double budget;
    {
        std::lock_guard<std::mutex> lo(c.opt_mu);
        budget = c.base_opt.serve_budget;
    }
    {
        // graph lookups only: the device may be busy
        std::lock_guard<std::mutex> lr(c.reg_mu);
        for (int32_t i = 0; i < count; ++i) {
            const gfr_query &q = queries[i];
            Ticket t;
            t.q = q;
            t.t_submit = Clock::now();
            auto git = c.graphs.find(q.graph);
            if (git == c.graphs.end()) {
                t.status = GFR_E_NOT_FOUND;
            } else {
                const Graph &g = *git->second;
                if ((q.kind != GFR_Q_BFS && q.kind != GFR_Q_SSSP) || q.source < 0 || q.source >= g.n ||
                    !q.out || q.reserved != 0 || (q.kind == GFR_Q_SSSP && !g.weighted)) {
                    t.status = GFR_E_INVALID;
                } else if ((double)session_bytes(c, g, q.kind) > budget) {
                    return GFR_E_CAPACITY;
                }
            }
            staged.push_back(t);
        }
    }
    Server &sv = server_of(c);
    {
        std::lock_guard<std::mutex> lk(sv.mu);
        for (int32_t i = 0; i < count; ++i) {
            const gfr_ticket id = sv.next++;
            Ticket &t = sv.tickets[id];
            t = staged[i];
            tickets_out[i] = id;
            if (t.status != GFR_OK) {   // completes at once with its error
                t.state = 2;
                t.t_done = Clock::now();
                sv.finished.push_back(id);
            } else {
                sv.queue.push_back(id);
            }
        }
    }
    sv.cv_work.notify_one();
    sv.cv_done.notify_all();
    return GFR_OK;
}

gfr_status gfr_poll(gfr_ctx *ctx, gfr_ticket *done, gfr_status *status, int32_t cap, int32_t *ndone,
                    int32_t timeout_us)
{
    if (!ctx || !ndone || cap < 0 || (cap > 0 && (!done || !status))) return GFR_E_INVALID;
    Ctx &c = *(Ctx *)ctx;
    Server &sv = server_of(c);
    std::unique_lock<std::mutex> lk(sv.mu);
    if (sv.finished.empty() && timeout_us > 0)
        sv.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !sv.finished.empty(); });
    int32_t k = 0;
    while (k < cap && !sv.finished.empty()) {
        const gfr_ticket t = sv.finished.front();
        sv.finished.pop_front();
        done[k] = t;
        status[k] = sv.tickets[t].status;
        sv.tickets.erase(t);
        ++k;
    }
    *ndone = k;
    return GFR_OK;
}

gfr_status gfr_cancel(gfr_ctx *ctx, gfr_ticket t)
{
    if (!ctx) return GFR_E_INVALID;
    Ctx &c = *(Ctx *)ctx;
    Server &sv = server_of(c);
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = std::find(sv.queue.begin(), sv.queue.end(), t);
    if (it == sv.queue.end()) return GFR_E_NOT_FOUND;   // unknown, running or finished
    sv.queue.erase(it);
    sv.tickets.erase(t);
    return GFR_OK;
}

}  // extern "C"
