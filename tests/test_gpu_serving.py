"""GPU tests of the serving runtime (submit / poll / cancel): every served
result equals the same query solved alone and the oracle, whatever batch it
ran in; admission, error and cancellation paths behave as the ABI states."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import paper_1501_05387_amd as gfr
    ctx = gfr.Context(0)
    graphs = {}
    for name, (row, col) in {"rmat12": graphgen.rmat(12), "grid64": graphgen.grid(64)}.items():
        w = graphgen.weights(row, col, 1000 if name.startswith("grid") else 64)
        graphs[name] = (row, col, w, ctx.graph_load_csr(row, col, w))
    yield gfr, ctx, graphs
    ctx.close()


def _drain(ctx, tickets, timeout=60.0):
    want = set(tickets)
    got = {}
    t0 = time.time()
    while want - set(got):
        for t, st in ctx.poll(64, 200000):
            got[t] = st
        assert time.time() - t0 < timeout, "serving did not finish"
    return got


def test_served_results_equal_alone_and_oracle(env):
    import torch
    gfr, ctx, graphs = env
    rng = np.random.default_rng(4)
    queries, outs, meta = [], [], []
    for i in range(150):
        name = ("rmat12", "grid64")[i % 3 == 0]
        row, col, w, g = graphs[name]
        kind = gfr.GFR_Q_BFS if rng.random() < 0.7 else gfr.GFR_Q_SSSP
        src = int(rng.integers(0, row.size - 1))
        out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
        queries.append((kind, g, src, out))
        outs.append(out)
        meta.append((name, kind, src))
    _say("serve mix", len(queries))
    tickets = []
    for i in range(0, len(queries), 25):            # arrivals in waves while earlier ones run
        tickets += ctx.submit_queries(queries[i:i + 25])
    got = _drain(ctx, tickets)
    assert all(st == gfr.GFR_OK for st in got.values())
    assert ctx.stat("serve.mean_batch") > 1.0
    for out, (name, kind, src) in zip(outs, meta):
        row, col, w, g = graphs[name]
        res = out.cpu().numpy()
        if kind == gfr.GFR_Q_BFS:
            assert np.array_equal(res, oracle.bfs(row, col, src))
            assert np.array_equal(res, ctx.bfs(g, src).cpu().numpy())
        else:
            assert np.array_equal(res.view(np.uint32), oracle.sssp(row, col, w, src))
            assert np.array_equal(res, ctx.sssp(g, src).cpu().numpy())
    assert ctx.stat("serve.p99_ms") >= ctx.stat("serve.p50_ms") > 0


def test_serving_host_outputs_and_one_at_a_time(env):
    gfr, ctx, graphs = env
    row, col, w, g = graphs["rmat12"]
    ctx.set_option("serve.max_batch", 1)
    try:
        outs = [np.empty(row.size - 1, np.int32) for _ in range(6)]
        qs = [(gfr.GFR_Q_SSSP if i % 2 else gfr.GFR_Q_BFS, g, 7 * i, outs[i]) for i in range(6)]
        ctx.stat("serve.reset")
        got = _drain(ctx, ctx.submit_queries(qs))
        assert all(st == gfr.GFR_OK for st in got.values())
        assert ctx.stat("serve.mean_batch") == 1.0
        for i, out in enumerate(outs):
            want = oracle.sssp(row, col, w, 7 * i) if i % 2 else oracle.bfs(row, col, 7 * i)
            assert np.array_equal(out.view(want.dtype), want)
    finally:
        ctx.set_option("serve.max_batch", 64)


def test_bad_queries_complete_with_errors(env):
    import torch
    gfr, ctx, graphs = env
    row, col, w, g = graphs["rmat12"]
    out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
    t_bad_src = ctx.submit_queries([(gfr.GFR_Q_BFS, g, row.size + 5, out)])[0]
    bogus = gfr.Graph(ctx, 987654, g.n, g.m, True)
    t_bad_graph = ctx.submit_queries([(gfr.GFR_Q_BFS, bogus, 0, out)])[0]
    got = _drain(ctx, [t_bad_src, t_bad_graph])
    assert got[t_bad_src] == gfr.GFR_E_INVALID
    assert got[t_bad_graph] == gfr.GFR_E_NOT_FOUND


def test_capacity_rejection(env):
    import torch
    gfr, ctx, graphs = env
    row, col, w, g = graphs["rmat12"]
    out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
    old = ctx.get_option("serve.budget_bytes")
    ctx.set_option("serve.budget_bytes", 1000)
    try:
        with pytest.raises(gfr.GfrError) as ei:
            ctx.submit_queries([(gfr.GFR_Q_BFS, g, 0, out)])
        assert ei.value.status == gfr.GFR_E_CAPACITY
    finally:
        ctx.set_option("serve.budget_bytes", old)


def test_admission_keeps_sessions_within_budget(env):
    """With a budget below the four (graph, kind) sessions of the mix, sessions
    are evicted and re-created as keys come and go, the resident footprint never
    exceeds the budget at any poll, and every result is still exact."""
    import torch
    gfr, ctx, graphs = env
    saved = {k: ctx.get_option(k) for k in ("serve.budget_bytes", "batch.min_bfs", "batch.min_sssp")}
    try:
        ctx.set_option("batch.min_bfs", 1)
        ctx.set_option("batch.min_sssp", 1)
        keys = [(name, kind) for name in ("rmat12", "grid64") for kind in (gfr.GFR_Q_BFS, gfr.GFR_Q_SSSP)]
        outs = {}
        for name, kind in keys:      # one query per key: all four sessions resident
            row, col, w, g = graphs[name]
            outs[(name, kind)] = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
            _drain(ctx, ctx.submit_queries([(kind, g, 1, outs[(name, kind)])]))
        full = ctx.stat("serve.session_bytes")
        budget = 0.6 * full
        ctx.set_option("serve.budget_bytes", budget)
        # the next pass of the runtime releases the idle sessions beyond the new budget
        name, kind = keys[0]
        _drain(ctx, ctx.submit_queries([(kind, graphs[name][3], 2, outs[(name, kind)])]))
        t0 = time.time()
        while ctx.stat("serve.session_bytes") > budget:
            assert time.time() - t0 < 10, "idle sessions beyond a lowered budget were kept"
            time.sleep(0.01)
        rng = np.random.default_rng(9)
        qs, meta = [], []
        for i in range(160):
            name, kind = keys[int(rng.integers(0, 4))]
            row, col, w, g = graphs[name]
            src = int(rng.integers(0, row.size - 1))
            out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
            qs.append((kind, g, src, out))
            meta.append((name, kind, src, out))
        _say("admission under budget", budget, "of", full)
        tickets = ctx.submit_queries(qs)
        want, got, t0 = set(tickets), {}, time.time()
        peak = 0.0
        while want - set(got):
            for t, st in ctx.poll(64, 20000):
                got[t] = st
            peak = max(peak, ctx.stat("serve.session_bytes"))
            assert ctx.stat("serve.session_bytes") <= budget
            assert time.time() - t0 < 90, "serving did not finish under the budget"
        assert all(got[t] == gfr.GFR_OK for t in tickets)
        for (name, kind, src, out) in meta[::8]:
            row, col, w, g = graphs[name]
            res = out.cpu().numpy()
            want_r = oracle.bfs(row, col, src) if kind == gfr.GFR_Q_BFS else oracle.sssp(row, col, w, src)
            assert np.array_equal(res.view(np.uint32) if kind == gfr.GFR_Q_SSSP else res, want_r)
        _say("peak resident session bytes", peak)
    finally:
        for k, v in saved.items():
            ctx.set_option(k, v)


def test_cancel_and_poll_timeout(env):
    import torch
    gfr, ctx, graphs = env
    row, col, w, g = graphs["grid64"]
    outs = [torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0") for _ in range(40)]
    tickets = ctx.submit_queries([(gfr.GFR_Q_SSSP, g, i, outs[i]) for i in range(40)])
    cancelled = None
    for t in reversed(tickets):
        try:
            ctx.cancel(t)
            cancelled = t
            break
        except gfr.GfrError as e:
            assert e.status == gfr.GFR_E_NOT_FOUND
    rest = [t for t in tickets if t != cancelled]
    got = _drain(ctx, rest)
    assert cancelled not in got
    assert all(st == gfr.GFR_OK for st in got.values())
    t0 = time.time()
    assert ctx.poll(8, 20000) == []
    assert time.time() - t0 >= 0.015
    with pytest.raises(gfr.GfrError) as ei:
        ctx.cancel(10 ** 12)
    assert ei.value.status == gfr.GFR_E_NOT_FOUND


def test_queries_join_running_sessions(env):
    """Queries submitted while a session is mid-traversal join it at a level
    boundary (continuous batching) and still equal the oracle; sessions of
    two graphs run side by side."""
    import torch
    gfr, ctx, graphs = env
    ctx.stat("serve.reset")
    ctx.set_option("batch.min_bfs", 1)      # batch from the first query on
    ctx.set_option("batch.min_sssp", 1)
    rng = np.random.default_rng(11)
    tickets, checks = [], []
    for wave in range(6):
        qs = []
        for i in range(8):
            name = "grid64" if i % 2 else "rmat12"
            row, col, w, g = graphs[name]
            kind = gfr.GFR_Q_SSSP if (i // 2) % 2 else gfr.GFR_Q_BFS
            src = int(rng.integers(0, row.size - 1))
            out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
            qs.append((kind, g, src, out))
            checks.append((name, kind, src, out))
        tickets += ctx.submit_queries(qs)
        time.sleep(0.002)                      # the next wave arrives mid-traversal
    got = _drain(ctx, tickets)
    ctx.set_option("batch.min_bfs", 8)
    ctx.set_option("batch.min_sssp", 24)
    assert all(st == gfr.GFR_OK for st in got.values())
    assert ctx.stat("serve.joined") > 0
    for name, kind, src, out in checks:
        row, col, w, g = graphs[name]
        want = oracle.bfs(row, col, src) if kind == gfr.GFR_Q_BFS else oracle.sssp(row, col, w, src)
        assert np.array_equal(out.cpu().numpy().view(want.dtype), want), (name, kind, src)


def test_graph_free_waits_for_its_queries(env):
    import torch
    gfr, ctx, graphs = env
    row, col = graphgen.rmat(10)
    w = graphgen.weights(row, col, 64)
    g = ctx.graph_load_csr(row, col, w)
    outs = [torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0") for _ in range(4)]
    tickets = ctx.submit_queries([(gfr.GFR_Q_SSSP, g, i, outs[i]) for i in range(4)])
    try:
        g.free()
        freed = True        # the queries finished before the call
    except gfr.GfrError as e:
        assert e.status == gfr.GFR_E_NOT_READY
        freed = False
    got = _drain(ctx, tickets)
    assert all(st == gfr.GFR_OK for st in got.values())
    for i, out in enumerate(outs):
        assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.sssp(row, col, w, i))
    if not freed:
        g.free()


@pytest.mark.parametrize("graphs", [0, 1])
def test_session_rounds_with_and_without_hipgraph(env, graphs):
    """Session rounds replayed from captured hipGraphs (many replays, with
    eager work and synchronisations between them) give the same results as
    plain launches and the oracle."""
    import torch
    gfr, ctx, graphs_ = env
    ctx.set_option("serve.hipgraph", graphs)
    ctx.set_option("batch.min_bfs", 1)
    ctx.set_option("batch.min_sssp", 1)
    try:
        rng = np.random.default_rng(20 + graphs)
        checks, tickets = [], []
        for wave in range(4):
            qs = []
            for i in range(12):
                name = ("rmat12", "grid64")[i % 2]
                row, col, w, g = graphs_[name]
                kind = (gfr.GFR_Q_BFS, gfr.GFR_Q_SSSP)[(i // 2) % 2]
                src = int(rng.integers(0, row.size - 1))
                out = torch.empty(row.size - 1, dtype=torch.int32, device="cuda:0")
                qs.append((kind, g, src, out))
                checks.append((name, kind, src, out))
            tickets += ctx.submit_queries(qs)
            torch.cuda.synchronize()                 # eager work between the replays
            _ = ctx.bfs(graphs_["rmat12"][3], wave)
        got = _drain(ctx, tickets)
        assert all(st == gfr.GFR_OK for st in got.values())
        for name, kind, src, out in checks:
            row, col, w, g = graphs_[name]
            want = oracle.bfs(row, col, src) if kind == gfr.GFR_Q_BFS else oracle.sssp(row, col, w, src)
            assert np.array_equal(out.cpu().numpy().view(want.dtype), want), (graphs, name, kind, src)
    finally:
        ctx.set_option("serve.hipgraph", 1)
        ctx.set_option("batch.min_bfs", 8)
        ctx.set_option("batch.min_sssp", 24)
