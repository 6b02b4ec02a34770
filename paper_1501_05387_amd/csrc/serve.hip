// serve.hip -- asynchronous query serving: submit / poll / cancel.
//
// A worker thread per context keeps a FIFO of submitted BFS / SSSP queries.
// Whenever the device is free it forms the next batch from the queue: the
// oldest admissible query fixes (graph, kind), and up to `serve.max_batch`
// (<= 64) queued queries of the same graph and kind join it in arrival order,
// as long as the batch's device footprint fits `serve.budget_bytes`.  Queries
// that arrive while a batch runs are picked up by the next one, so the batch
// size follows the load.  A batch runs through the batched kernels (one
// traversal for up to 64 sources, msbfs.hip / sssp_batch.hip); each query's
// row is then copied to its own output buffer and its ticket completes.
//
// Footprints follow the memory the batched solvers take per vertex and edge;
// a query whose smallest batch (itself alone) cannot fit the budget is
// rejected at submission with GFR_E_CAPACITY.
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

struct Server {
    Ctx *ctx = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<gfr_ticket> queue;
    std::unordered_map<gfr_ticket, Ticket> tickets;
    std::deque<gfr_ticket> finished;
    bool stop = false;
    gfr_ticket next = 1;
    // statistics
    std::vector<double> latency_ms;
    uint64_t batches = 0, batched_queries = 0;
    DevMem stage;   // [k][n] results of the running batch
};

// Device bytes a batch of k queries of `kind` on g holds (state + staging).
static uint64_t batch_footprint(const Graph &g, int32_t kind, int32_t k)
{
    const uint64_t n = (uint64_t)g.n, nw = ((n + 63) / 64) * 2;
    const uint64_t queue = 12 * n + 4 * ((uint64_t)g.m / 1024 + 2);
    uint64_t state;
    if (kind == GFR_Q_BFS) state = 24 * n + 32 * nw + queue;
    else state = 256 * n + 8 * n + 128 * n + 64 * nw + queue;
    return state + 4 * n * (uint64_t)k + (1u << 20);
}

static void worker_loop(Server *sv)
{
    Ctx &c = *sv->ctx;
    for (;;) {
        std::vector<gfr_ticket> batch;
        int64_t gh = 0;
        int32_t kind = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->stop) return;
        }
        // lock order everywhere: context mutex, then server mutex
        std::unique_lock<std::recursive_mutex> lc(c.mu);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->stop) return;
            if (sv->queue.empty()) continue;   // cancelled meanwhile
            const double budget = c.opt.serve_budget;
            const int32_t maxb = std::max(1, std::min(64, c.opt.serve_max_batch));
            const gfr_ticket head = sv->queue.front();
            gh = sv->tickets[head].q.graph;
            kind = sv->tickets[head].q.kind;
            for (auto it = sv->queue.begin(); it != sv->queue.end() && (int32_t)batch.size() < maxb;) {
                Ticket &t = sv->tickets[*it];
                if (t.q.graph == gh && t.q.kind == kind) {
                    batch.push_back(*it);
                    it = sv->queue.erase(it);
                } else {
                    ++it;
                }
            }
            // admission by footprint (the graph may have been freed meanwhile)
            auto git = c.graphs.find(gh);
            if (git != c.graphs.end()) {
                while (batch.size() > 1 &&
                       (double)batch_footprint(*git->second, kind, (int32_t)batch.size()) > budget) {
                    sv->queue.push_front(batch.back());
                    batch.pop_back();
                }
            }
            for (auto t : batch) sv->tickets[t].state = 1;
        }
        gfr_status st = GFR_OK;
        std::string err;
        {
            try {
                GFR_HIP(hipSetDevice(c.device));
                Graph &g = get_graph(c, gh);
                OptScope os(c, g);
                const int32_t k = (int32_t)batch.size();
                std::vector<int32_t> src(k);
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    for (int32_t i = 0; i < k; ++i) src[i] = sv->tickets[batch[i]].q.source;
                }
                const size_t row = 4ull * g.n;
                if (sv->stage.bytes < row * k) sv->stage.alloc(row * k);
                hipStream_t s = c.stream;
                c.stats.clear();
                c.ktimer.on = false;
                // a lone query runs on the single-source solver, which needs
                // no per-source masks or rows
                if (kind == GFR_Q_BFS) {
                    if (k == 1) run_bfs(c, g, src[0], sv->stage.as<int32_t>(), s);
                    else run_bfs_batch(c, g, src.data(), k, sv->stage.as<int32_t>(), s);
                } else {
                    if (k == 1) run_sssp(c, g, src[0], sv->stage.as<uint32_t>(), s);
                    else run_sssp_batch(c, g, src.data(), k, sv->stage.as<uint32_t>(), s);
                }
                for (int32_t i = 0; i < k; ++i) {
                    gfr_query q;
                    {
                        std::lock_guard<std::mutex> lk(sv->mu);
                        q = sv->tickets[batch[i]].q;
                    }
                    if (q.out_on_device)
                        GFR_HIP(hipMemcpyAsync(q.out, (char *)sv->stage.p + row * i, row, hipMemcpyDeviceToDevice, s));
                    else
                        copy_to_host(c, q.out, (char *)sv->stage.p + row * i, row, s);
                }
                GFR_HIP(hipStreamSynchronize(s));
            } catch (const Error &e) {
                st = e.code;
                err = e.msg;
            } catch (...) {
                st = GFR_E_DEVICE;
            }
        }
        lc.unlock();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            const auto now = Clock::now();
            for (auto t : batch) {
                Ticket &tk = sv->tickets[t];
                tk.state = 2;
                tk.status = st;
                tk.t_done = now;
                sv->latency_ms.push_back(std::chrono::duration<double, std::milli>(now - tk.t_submit).count());
                sv->finished.push_back(t);
            }
            sv->batches += 1;
            sv->batched_queries += batch.size();
        }
        sv->cv_done.notify_all();
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
    if (sv->worker.joinable()) sv->worker.join();
    delete sv;
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
    }
    return *c.server;
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
    std::lock_guard<std::mutex> lk(sv.mu);
    if (key == "serve.completed") *value = (double)sv.latency_ms.size();
    else if (key == "serve.batches") *value = (double)sv.batches;
    else if (key == "serve.mean_batch") *value = sv.batches ? (double)sv.batched_queries / sv.batches : 0.0;
    else if (key == "serve.p50_ms") *value = percentile(sv.latency_ms, 50);
    else if (key == "serve.p99_ms") *value = percentile(sv.latency_ms, 99);
    else if (key == "serve.queued") *value = (double)sv.queue.size();
    else if (key == "serve.reset") {
        sv.latency_ms.clear();
        sv.batches = sv.batched_queries = 0;
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
    {
        // graph lookups only: the device may be busy with a running batch
        std::lock_guard<std::mutex> lr(c.reg_mu);
        const double budget = c.opt.serve_budget;
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
                } else if ((double)batch_footprint(g, q.kind, 1) > budget) {
                    return GFR_E_CAPACITY;
                }
            }
            staged.push_back(t);
        }
    }
    Server *svp = &server_of(c);
    Server &sv = *svp;
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
