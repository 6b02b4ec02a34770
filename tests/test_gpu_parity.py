"""GPU parity: the HIP engine (through the C ABI) against the CPU oracle on the
same seeded inputs.  BFS depths, SSSP distances and CC labels must match bit
for bit; BC within 1e-5 relative; FP32 PageRank within 1e-6 L1 of the FP64
oracle run for the same number of iterations.

Sizes span several load-balancing chunks and ragged tails; the edge cases
cover isolated and degree-zero sources, hubs larger than one chunk, graphs
without edges, many components and long thin frontiers.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_05387_amd as gfr
    c = gfr.Context(0)
    yield c
    c.close()


def _host(t):
    import torch
    if isinstance(t, torch.Tensor):
        return t.cpu().numpy()
    return t


def _load(ctx, row, col, w=None):
    return ctx.graph_load_csr(row, col, w)


def _star(k):
    return graphgen.from_edges(k + 1, np.zeros(k, np.int32), np.arange(1, k + 1))


def _path(n):
    return graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n))


GRAPHS = {
    "rmat12": lambda: graphgen.rmat(12),
    "rmat16": lambda: graphgen.rmat(16),
    "grid96": lambda: graphgen.grid(96),
    "star5000": lambda: _star(5000),
    "path3000": lambda: _path(3000),
    "forest": lambda: graphgen.from_edges(2000, np.arange(0, 1998, 2), np.arange(1, 1999, 2)),
}

_cache = {}


def graph(name):
    if name not in _cache:
        row, col = GRAPHS[name]()
        w = graphgen.weights(row, col, 1000 if name.startswith("grid") else 64)
        _cache[name] = (row, col, w)
    return _cache[name]


def _sources(row, col, k, seed=3):
    n = row.size - 1
    try:
        s = list(graphgen.sample_sources(row, col, min(k, 4), seed=seed))
    except ValueError:
        s = []
    s += [0, n - 1]
    deg = np.diff(row)
    iso = np.nonzero(deg == 0)[0]
    if iso.size:
        s.append(int(iso[0]))
    return sorted(set(int(x) for x in s))


# -------------------------------------------------------------------- BFS
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_bfs_matches_oracle(ctx, name, direction):
    row, col, w = graph(name)
    g = _load(ctx, row, col)
    ctx.set_option("bfs.direction", direction)
    try:
        for s in _sources(row, col, 4):
            _say("bfs", name, "dir", direction, "src", s)
            got = _host(ctx.bfs(g, s))
            want = oracle.bfs(row, col, s)
            assert np.array_equal(got, want), (name, direction, s, int(np.sum(got != want)))
    finally:
        ctx.set_option("bfs.direction", 0)
        g.free()


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("frontier", [1, 2])
def test_bfs_frontier_representations(ctx, name, frontier):
    """Queue levels (advance + compaction) and mark-byte levels (one launch per
    level) give the oracle's depths on every graph, whichever the graph class."""
    row, col, w = graph(name)
    g = _load(ctx, row, col)
    ctx.set_option("bfs.frontier", frontier)
    try:
        for s in _sources(row, col, 4):
            _say("bfs", name, "frontier", frontier, "src", s)
            got = _host(ctx.bfs(g, s))
            want = oracle.bfs(row, col, s)
            assert np.array_equal(got, want), (name, frontier, s, int(np.sum(got != want)))
            if frontier == 2:
                assert ctx.stat("levels") == int(want.max()) + 1 and ctx.stat("pull_levels") == 0
    finally:
        ctx.set_option("bfs.frontier", 0)
        g.free()


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("mapping,threshold", [(2, 4096), (0, 4096), (0, 64)])
def test_bfs_push_work_mappings(ctx, name, mapping, threshold):
    """Push levels with the per-vertex mapping of Sec. 4.4 (lists of a
    work-group's size or more by the whole work-group, of 64 or more by a wave,
    the rest per thread) alone, and the hybrid that uses it below a frontier
    size and equal edge chunks above it, give the oracle's depths.  The star's
    centre (5000 edges) takes the work-group path, R-MAT hubs the wave path."""
    row, col, w = graph(name)
    g = _load(ctx, row, col)
    ctx.set_option("bfs.direction", 1)
    ctx.set_option("bfs.frontier", 1)
    ctx.set_option("advance.mapping", mapping)
    ctx.set_option("advance.twc_threshold", threshold)
    try:
        for s in _sources(row, col, 4):
            _say("bfs push mapping", mapping, "threshold", threshold, name, "src", s)
            got = _host(ctx.bfs(g, s))
            want = oracle.bfs(row, col, s)
            assert np.array_equal(got, want), (name, mapping, threshold, s, int(np.sum(got != want)))
    finally:
        ctx.set_option("bfs.direction", 0)
        ctx.set_option("bfs.frontier", 0)
        ctx.set_option("advance.mapping", 1)
        ctx.set_option("advance.twc_threshold", 4096)
        g.free()


def test_bfs_rmat16_from_vertex0_all_chunks(ctx):
    row, col, _ = graph("rmat16")
    g = _load(ctx, row, col)
    want = oracle.bfs(row, col, 0)
    try:
        for ch in (256, 512, 1024, 2048, 4096):
            ctx.set_option("advance.chunk", ch)
            _say("bfs rmat16 src0 chunk", ch)
            assert np.array_equal(_host(ctx.bfs(g, 0)), want)
    finally:
        ctx.set_option("advance.chunk", 1024)
        g.free()


def test_bfs_host_output_and_stats(ctx):
    row, col, _ = graph("rmat12")
    g = _load(ctx, row, col)
    out = np.empty(row.size - 1, np.int32)
    ctx.bfs(g, 0, out=out)
    assert np.array_equal(out, oracle.bfs(row, col, 0))
    assert ctx.stat("levels") >= 2
    assert ctx.stat("kernel_ms") > 0
    g.free()


# ------------------------------------------------------------------- SSSP
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("delta", [0, 1, 7, 100000])
@pytest.mark.parametrize("frontier", [1, 2])
def test_sssp_matches_oracle(ctx, name, delta, frontier):
    """Queue iterations (advance + compaction) and mark-byte iterations (one
    launch each, near/far sets as bytes) give the oracle's distances on every
    graph, for bucket widths from 1 (many splits) to one bucket."""
    row, col, w = graph(name)
    g = _load(ctx, row, col, w)
    ctx.set_option("sssp.delta", delta)
    ctx.set_option("sssp.frontier", frontier)
    try:
        for s in _sources(row, col, 4):
            _say("sssp", name, "delta", delta, "frontier", frontier, "src", s)
            got = _host(ctx.sssp(g, s)).view(np.uint32)
            want = oracle.sssp(row, col, w, s)
            assert np.array_equal(got, want), (name, delta, frontier, s, int(np.sum(got != want)))
    finally:
        ctx.set_option("sssp.delta", 0)
        ctx.set_option("sssp.frontier", 0)
        g.free()


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("alpha", [24, 1e6])
@pytest.mark.parametrize("delta", [0, 1])
def test_sssp_pull_directions(ctx, name, alpha, delta):
    """Direction-optimizing single-source SSSP: iterations whose near queue
    carries more than m / alpha edges relax by a pull sweep (alpha 1e6: nearly
    every iteration after the first pulls).  Distances equal the oracle's with
    one bucket and with many (delta 1)."""
    row, col, w = graph(name)
    g = _load(ctx, row, col, w)
    ctx.set_option("sssp.pull_alpha", alpha)
    ctx.set_option("sssp.delta", delta)
    try:
        pulls = 0
        for s in _sources(row, col, 4):
            _say("sssp pull", name, "alpha", alpha, "delta", delta, "src", s)
            got = _host(ctx.sssp(g, s)).view(np.uint32)
            want = oracle.sssp(row, col, w, s)
            assert np.array_equal(got, want), (name, alpha, delta, s, int(np.sum(got != want)))
            pulls += ctx.stat("pull_iterations")
        if alpha == 1e6 and name in ("rmat16", "grid96"):
            assert pulls >= 1
    finally:
        ctx.set_option("sssp.pull_alpha", 0)
        ctx.set_option("sssp.delta", 0)
        g.free()


def test_sssp_chunks(ctx):
    row, col, w = graph("rmat16")
    g = _load(ctx, row, col, w)
    want = oracle.sssp(row, col, w, 0)
    try:
        for ch in (256, 4096):
            ctx.set_option("advance.chunk", ch)
            _say("sssp rmat16 chunk", ch)
            assert np.array_equal(_host(ctx.sssp(g, 0)).view(np.uint32), want)
    finally:
        ctx.set_option("advance.chunk", 1024)
        g.free()


@pytest.mark.parametrize("frontier", [1, 2])
def test_sssp_rejects_unweighted_and_overflow(ctx, frontier):
    import paper_1501_05387_amd as gfr
    row, col = _path(10)
    g = _load(ctx, row, col)
    with pytest.raises(gfr.GfrError):
        ctx.sssp(g, 0)
    g.free()
    w = np.full(col.size, 0x7FFFFFFF, np.uint32)
    g = _load(ctx, row, col, w)
    ctx.set_option("sssp.frontier", frontier)
    try:
        with pytest.raises(gfr.GfrError) as ei:
            ctx.sssp(g, 0)
        assert ei.value.status == gfr.GFR_E_INVALID
        # the largest distance that fits: 0x7FFFFFFF + 0x7FFFFFFF = 0xFFFFFFFE on a 3-vertex path (the
        # relaxation back from the far end sums past 32 bits and is not an improvement)
        row3, col3 = _path(3)
        w3 = np.full(col3.size, 0x7FFFFFFF, np.uint32)
        g3 = _load(ctx, row3, col3, w3)
        got = _host(ctx.sssp(g3, 0)).view(np.uint32)
        assert got.tolist() == [0, 0x7FFFFFFF, 0xFFFFFFFE] == oracle.sssp(row3, col3, w3, 0).tolist()
        # batched, with 32-bit rows (whole rows and lane-per-edge groups) and
        # with narrow rows tried first
        ctx.set_option("batch.min_sssp", 1)
        for narrow, sparse in ((0, 0), (0, 8), (3, 8)):
            ctx.set_option("batch.narrow", narrow)
            ctx.set_option("batch.sparse", sparse)
            src = np.array([0, 2, 1], np.int32)
            b = _host(ctx.sssp_batch(g3, src)).view(np.uint32).reshape(3, 3)
            for i in range(3):
                assert np.array_equal(b[i], oracle.sssp(row3, col3, w3, int(src[i]))), (narrow, sparse, i)
            with pytest.raises(gfr.GfrError) as ei:
                ctx.sssp_batch(g, np.array([0, 9], np.int32))
            assert ei.value.status == gfr.GFR_E_INVALID
        g3.free()
    finally:
        ctx.set_option("batch.sparse", 8)
        ctx.set_option("sssp.frontier", 0)
        ctx.set_option("batch.min_sssp", 24)
        ctx.set_option("batch.narrow", 0)
        g.free()


# ----------------------------------------------------------- predecessors
@pytest.mark.parametrize("name", list(GRAPHS))
def test_predecessors_match_oracle(ctx, name):
    row, col, w = graph(name)
    g = _load(ctx, row, col, w)
    for s in _sources(row, col, 3):
        _say("pred", name, "source", s)
        d, p = ctx.bfs(g, s, pred=True)
        do, po = oracle.bfs_pred(row, col, s)
        assert np.array_equal(_host(d), do) and np.array_equal(_host(p), po)
        d, p = ctx.sssp(g, s, pred=True)
        do, po = oracle.sssp_pred(row, col, w, s)
        assert np.array_equal(_host(d).view(np.uint32), do) and np.array_equal(_host(p), po)
    g.free()


def test_predecessors_host_outputs_and_default(ctx):
    row, col, w = graph("star5000")
    n = row.size - 1
    g = _load(ctx, row, col, w)
    dh, ph = np.empty(n, np.int32), np.empty(n, np.int32)
    d, p = ctx.bfs(g, 4321, out=dh, pred=ph)       # the centre's row (5000 entries) takes the wave path
    assert d is dh and p is ph
    do, po = oracle.bfs_pred(row, col, 4321)
    assert np.array_equal(dh, do) and np.array_equal(ph, po) and ph[0] == 4321
    sh = np.empty(n, np.uint32)
    ctx.sssp(g, 4321, out=sh, pred=ph)
    so, po = oracle.sssp_pred(row, col, w, 4321)
    assert np.array_equal(sh, so) and np.array_equal(ph, po)
    assert not isinstance(ctx.bfs(g, 0), tuple)     # no predecessors unless asked
    g.free()


# --------------------------------------------------------------------- CC
@pytest.mark.parametrize("name", list(GRAPHS))
def test_cc_matches_oracle(ctx, name):
    row, col, _ = graph(name)
    g = _load(ctx, row, col)
    _say("cc", name)
    lab, k = ctx.cc(g)
    want, kw = oracle.cc(row, col)
    assert np.array_equal(_host(lab), want)
    assert k == kw
    g.free()


# --------------------------------------------------------------------- PR
@pytest.mark.parametrize("name", ["rmat12", "rmat16", "grid96", "star5000", "forest"])
def test_pagerank_matches_oracle(ctx, name):
    row, col, _ = graph(name)
    g = _load(ctx, row, col)
    _say("pagerank", name)
    x, it, l1 = ctx.pagerank(g, 0.85, 1e-6, 1000)
    x = _host(x).astype(np.float64)
    xo, ito, _ = oracle.pagerank(row, col, 0.85, 0.0, it)      # the oracle at the GPU's iteration count
    err = np.abs(x - xo).sum()
    _say("pagerank", name, "iters", it, "L1 err", err)
    assert err <= 1e-6, err
    assert abs(x.sum() - 1.0) < 1e-5
    assert l1 < 1e-6 and it < 1000
    _, it_ref, _ = oracle.pagerank(row, col, 0.85, 1e-6, 1000)
    assert abs(it - it_ref) <= 1
    g.free()


def test_pagerank_max_iter(ctx):
    row, col, _ = graph("rmat12")
    g = _load(ctx, row, col)
    x, it, l1 = ctx.pagerank(g, 0.85, 0.0, 5)
    assert it == 5
    xo, _, _ = oracle.pagerank(row, col, 0.85, 0.0, 5)
    assert np.abs(_host(x) - xo).sum() <= 1e-6
    g.free()


# --------------------------------------------------------------------- BC
@pytest.mark.parametrize("name", ["rmat12", "grid96", "star5000", "path3000", "forest"])
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_bc_matches_oracle(ctx, name, direction):
    row, col, _ = graph(name)
    n = row.size - 1
    src = np.array(_sources(row, col, 4)[:6], np.int32)
    g = _load(ctx, row, col)
    _say("bc", name, "direction", direction, "sources", src.tolist())
    ctx.set_option("bc.direction", direction)
    try:
        got = _host(ctx.bc(g, src)).astype(np.float64)
    finally:
        ctx.set_option("bc.direction", 0)
    want = oracle.bc(row, col, src)
    nz = want != 0
    rel = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert np.all(got[~nz] == 0)
    assert rel.size == 0 or rel.max() <= 1e-5, rel.max()
    g.free()


def test_bc_directions_agree_bitwise(ctx):
    """The forward discovery direction changes neither a level nor the order of
    any sum, so push-only, pull-only and automatic runs agree bit for bit."""
    row, col, _ = graph("rmat16")
    src = np.array(_sources(row, col, 4)[:5], np.int32)
    g = _load(ctx, row, col)
    out = {}
    try:
        for d in (1, 2, 0):
            ctx.set_option("bc.direction", d)
            out[d] = _host(ctx.bc(g, src)).copy()
            if d == 0:
                assert ctx.stat("pull_levels") > 0 and ctx.stat("push_levels") > 0
    finally:
        ctx.set_option("bc.direction", 0)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    g.free()


def test_bc_rejects_duplicates(ctx):
    import paper_1501_05387_amd as gfr
    row, col, _ = graph("rmat12")
    g = _load(ctx, row, col)
    with pytest.raises(gfr.GfrError):
        ctx.bc(g, [1, 1])
    g.free()


# ------------------------------------------------------------ edge cases
def test_graph_without_edges(ctx):
    row = np.zeros(6, np.int32)
    col = np.zeros(0, np.int32)
    g = ctx.graph_load_csr(row, col, np.zeros(0, np.uint32))
    d = _host(ctx.bfs(g, 2))
    assert d.tolist() == [-1, -1, 0, -1, -1]
    s = _host(ctx.sssp(g, 4)).view(np.uint32)
    assert s[4] == 0 and np.all(s[:4] == 0xFFFFFFFF)
    lab, k = ctx.cc(g)
    assert _host(lab).tolist() == list(range(5)) and k == 5
    x, it, _ = ctx.pagerank(g)
    assert np.allclose(_host(x), 0.2)
    g.free()


def test_single_vertex(ctx):
    g = ctx.graph_load_csr(np.zeros(2, np.int32), np.zeros(0, np.int32))
    assert _host(ctx.bfs(g, 0)).tolist() == [0]
    assert _host(ctx.bc(g, [0])).tolist() == [0.0]
    g.free()


def test_bad_arguments(ctx):
    import paper_1501_05387_amd as gfr
    row, col, _ = graph("rmat12")
    g = _load(ctx, row, col)
    for call in (lambda: ctx.bfs(g, -1), lambda: ctx.bfs(g, row.size - 1),
                 lambda: ctx.pagerank(g, 1.5), lambda: ctx.set_option("nope", 1),
                 lambda: ctx.set_option("advance.chunk", 300)):
        with pytest.raises(gfr.GfrError) as ei:
            call()
        assert ei.value.status == gfr.GFR_E_INVALID
    g.free()
    with pytest.raises(gfr.GfrError) as ei:
        ctx.bfs(g, 0)
    assert ei.value.status == gfr.GFR_E_NOT_FOUND


def test_determinism(ctx):
    row, col, w = graph("rmat16")
    g = _load(ctx, row, col, w)
    a = [_host(ctx.sssp(g, 5)).copy() for _ in range(2)]
    assert np.array_equal(a[0], a[1])
    p = [_host(ctx.pagerank(g)[0]).copy() for _ in range(2)]
    assert np.array_equal(p[0], p[1])
    l = [_host(ctx.cc(g)[0]).copy() for _ in range(2)]
    assert np.array_equal(l[0], l[1])
    g.free()


# ---------------------------------------------------------------- batching
def test_batch_equals_single(ctx):
    row, col, w = graph("rmat12")
    n = row.size - 1
    g = _load(ctx, row, col, w)
    src = np.array([0, 5, 5, 17, n - 1], np.int32)
    _say("bfs_batch / sssp_batch")
    d = _host(ctx.bfs_batch(g, src)).reshape(len(src), n)
    s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(len(src), n)
    for i, x in enumerate(src):
        assert np.array_equal(d[i], oracle.bfs(row, col, x))
        assert np.array_equal(s[i], oracle.sssp(row, col, w, x))
    g.free()


@pytest.mark.parametrize("name", ["rmat12", "grid96", "star5000", "path3000", "forest"])
@pytest.mark.parametrize("k", [1, 64, 70])
def test_batch_many_sources(ctx, name, k):
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(k)
    src = rng.integers(0, n, size=k).astype(np.int32)
    src[0] = 0
    if k > 2:
        src[1] = src[2]                                  # a duplicated source
        iso = np.nonzero(np.diff(row) == 0)[0]
        if iso.size:
            src[-1] = iso[0]                             # an isolated source
    g = _load(ctx, row, col, w)
    _say("batch", name, "k", k)
    for mb in (1, 10 ** 6):      # shared traversal for every k, then sequential solves
        ctx.set_option("batch.min_bfs", mb)
        ctx.set_option("batch.min_sssp", mb)
        d = _host(ctx.bfs_batch(g, src)).reshape(k, n)
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(k, n)
        if mb == 1:
            d1, s1 = d.copy(), s.copy()
    ctx.set_option("batch.min_bfs", 8)
    ctx.set_option("batch.min_sssp", 24)
    assert np.array_equal(d, d1) and np.array_equal(s, s1)
    for i in range(0, k, max(1, k // 9)):
        assert np.array_equal(d[i], oracle.bfs(row, col, src[i])), (name, k, i)
        assert np.array_equal(s[i], oracle.sssp(row, col, w, src[i])), (name, k, i)
    assert np.array_equal(d[-1], oracle.bfs(row, col, src[-1]))
    assert np.array_equal(s[-1], oracle.sssp(row, col, w, src[-1]))
    g.free()


@pytest.mark.parametrize("delta", [1, 50, 1 << 30])
def test_sssp_batch_buckets(ctx, delta):
    row, col, w = graph("grid96")
    n = row.size - 1
    src = np.arange(0, n, n // 40, dtype=np.int32)[:40]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.delta", delta)
    ctx.set_option("batch.min_sssp", 1)
    try:
        _say("sssp_batch grid96 delta", delta)
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(len(src), n)
        for i in (0, 7, 39):
            assert np.array_equal(s[i], oracle.sssp(row, col, w, src[i]))
    finally:
        ctx.set_option("batch.delta", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("name", ["rmat16", "grid96", "star5000", "path3000", "forest"])
@pytest.mark.parametrize("delta", [0, 50])
@pytest.mark.parametrize("narrow", [0, 3])
def test_sssp_batch_pending_queries(ctx, name, delta, narrow):
    """A queued vertex also relaxes the queries improved at it earlier in the
    same launch (batch.pending 1, the default) or only its queued ones (0):
    the oracle's distances on every row either way, with one bucket and narrow
    buckets, 32-bit rows and narrow rows from 8 bits, a full and a ragged
    batch."""
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(13)
    src = rng.integers(0, n, size=70).astype(np.int32)
    src[0] = 0
    src[5] = src[6]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.min_sssp", 1)
    ctx.set_option("batch.delta", delta)
    ctx.set_option("batch.narrow", narrow)
    try:
        ref = [oracle.sssp(row, col, w, int(x)) for x in src]
        visits = []
        for pending in (1, 0):
            ctx.set_option("batch.pending", pending)
            _say("sssp_batch pending", pending, name, "delta", delta, "narrow", narrow)
            got = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, n)
            visits.append(ctx.stat("relaxations"))
            for i in range(src.size):
                assert np.array_equal(got[i], ref[i]), (name, pending, delta, narrow, i)
        print("edge visits with / without pending queries:", visits)
    finally:
        ctx.set_option("batch.pending", 1)
        ctx.set_option("batch.narrow", 0)
        ctx.set_option("batch.delta", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("name", ["rmat16", "grid96", "star5000", "path3000", "forest"])
@pytest.mark.parametrize("delta", [0, 50])
@pytest.mark.parametrize("pending", [1, 0])
def test_sssp_batch_sparse_groups(ctx, name, delta, pending):
    """Groups of edges with few queries each are relaxed one lane per edge
    (batch.sparse): the oracle's distances on every row with every group in
    that form (64), with a low threshold (2), the default (8) and none (0), with one
    bucket and narrow buckets (far marks written lane by lane), a full and a
    ragged batch."""
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(17)
    src = rng.integers(0, n, size=70).astype(np.int32)
    src[0] = 0
    src[5] = src[6]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.min_sssp", 1)
    ctx.set_option("batch.delta", delta)
    ctx.set_option("batch.pending", pending)
    try:
        ref = [oracle.sssp(row, col, w, int(x)) for x in src]
        for sparse in (64, 2, 8, 0):
            ctx.set_option("batch.sparse", sparse)
            _say("sssp_batch sparse", sparse, name, "delta", delta, "pending", pending)
            got = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, n)
            for i in range(src.size):
                assert np.array_equal(got[i], ref[i]), (name, sparse, delta, pending, i)
    finally:
        ctx.set_option("batch.sparse", 8)
        ctx.set_option("batch.pending", 1)
        ctx.set_option("batch.delta", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("name", ["rmat16", "grid96", "star5000", "path3000", "forest"])
@pytest.mark.parametrize("delta", [0, 50])
def test_sssp_batch_pair_kernel(ctx, name, delta):
    """32-bit rows relaxed two edges per row load (batch.pair 1: each half-wave
    one edge, two queries per lane) and one edge per load (batch.pair 0) give
    the oracle's distances on every row, with one bucket and with narrow
    buckets (far marks); 70 queries make a full and a ragged batch, and a hub
    (the star's centre) exercises groups that leave one vertex."""
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(11)
    src = rng.integers(0, n, size=70).astype(np.int32)
    src[0] = 0
    src[5] = src[6]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.min_sssp", 1)
    ctx.set_option("batch.delta", delta)
    try:
        ref = [oracle.sssp(row, col, w, int(x)) for x in src]
        outs = []
        for pair in (1, 0):
            ctx.set_option("batch.pair", pair)
            _say("sssp_batch pair", pair, name, "delta", delta)
            got = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, n)
            for i in range(src.size):
                assert np.array_equal(got[i], ref[i]), (name, pair, delta, i)
            outs.append(got)
        assert np.array_equal(outs[0], outs[1])
    finally:
        ctx.set_option("batch.pair", 0)
        ctx.set_option("batch.delta", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


def test_kernel_timing_modes(ctx):
    """profile.kernels 1 times every level launch, 2 only the advance kernels
    (the compactions run untimed); the results do not change."""
    row, col, w = graph("rmat16")
    srcs = graphgen.sample_sources(row, col, 64)
    g = _load(ctx, row, col, w)
    try:
        got = {}
        for mode in (0, 1, 2):
            ctx.set_option("profile.kernels", mode)
            _say("kernel timing mode", mode)
            got[mode] = _host(ctx.sssp_batch(g, srcs)).view(np.uint32)
            def st(key):
                try:
                    return ctx.stat(key)
                except Exception:   # a statistic the call did not produce
                    return 0.0
            relax, compact = st("t.bsssp_relax.n"), st("t.bsssp_compact.n")
            if mode == 0:
                assert relax == 0 and compact == 0
            elif mode == 1:
                assert relax > 0 and compact > 0
            else:
                assert relax > 0 and compact == 0 and st("t.bsssp_relax.ms") > 0
        assert np.array_equal(got[0], got[1]) and np.array_equal(got[0], got[2])
        n = row.size - 1
        assert np.array_equal(got[2].reshape(64, n)[5], oracle.sssp(row, col, w, int(srcs[5])))
    finally:
        ctx.set_option("profile.kernels", 0)
        g.free()


def test_step_graph_replays(ctx):
    """graph.steps 1: the level loops replay captured hipGraphs of their level
    launches.  Each solver runs four times into the same buffers (one capture,
    then replays), with eager work and synchronisations between the calls;
    every replay equals the plain launches and the oracle."""
    import torch
    row, col, w = graph("rmat16")
    n = row.size - 1
    srcs = graphgen.sample_sources(row, col, 64)
    g = _load(ctx, row, col, w)
    dev = "cuda:0"
    outs = {"bfs": torch.empty(n, dtype=torch.int32, device=dev), "sssp": torch.empty(n, dtype=torch.int32, device=dev),
            "bfs_batch": torch.empty(64 * n, dtype=torch.int32, device=dev),
            "sssp_batch": torch.empty(64 * n, dtype=torch.int32, device=dev)}
    calls = {"bfs": lambda o: ctx.bfs(g, int(srcs[0]), out=o), "sssp": lambda o: ctx.sssp(g, int(srcs[0]), out=o),
             "bfs_batch": lambda o: ctx.bfs_batch(g, srcs, out=o), "sssp_batch": lambda o: ctx.sssp_batch(g, srcs, out=o)}
    try:
        ctx.set_option("graph.steps", 0)
        plain = {}
        for k, f in calls.items():
            f(outs[k])
            plain[k] = outs[k].clone()
        assert np.array_equal(plain["bfs"].cpu().numpy(), oracle.bfs(row, col, int(srcs[0])))
        assert np.array_equal(plain["sssp"].cpu().numpy().view(np.uint32), oracle.sssp(row, col, w, int(srcs[0])))
        ctx.set_option("graph.steps", 1)
        junk = torch.zeros(1 << 20, device=dev)
        for rep in range(4):
            for k, f in calls.items():
                outs[k].fill_(-7)
                junk.add_(1.0)   # eager work of the program between the replays
                torch.cuda.synchronize()
                f(outs[k])
                replays = ctx.stat("graph_launches")
                _say("step graphs", k, "call", rep, "graph launches", replays)
                assert replays >= 1, k
                assert torch.equal(outs[k], plain[k]), (k, rep)
    finally:
        ctx.set_option("graph.steps", 0)
        g.free()


@pytest.mark.parametrize("alpha", [1e-6, 24, 1e9])
def test_bfs_batch_directions(ctx, alpha):
    row, col, _ = graph("rmat16")
    n = row.size - 1
    src = graphgen.sample_sources(row, col, 64)
    g = _load(ctx, row, col)
    ctx.set_option("msbfs.alpha", alpha)
    try:
        _say("bfs_batch rmat16 alpha", alpha)
        d = _host(ctx.bfs_batch(g, src)).reshape(64, n)
        for i in (0, 31, 63):
            assert np.array_equal(d[i], oracle.bfs(row, col, src[i]))
    finally:
        ctx.set_option("msbfs.alpha", 4)
        g.free()


def test_host_outputs_span_several_bounce_chunks(ctx):
    """Batched results written to pageable (numpy) and pinned (torch) host
    memory equal the device results; 64 x 2^18 x 4 bytes spans three 32 MiB
    bounce chunks, the last one ragged."""
    import torch
    row, col = graphgen.rmat(18)
    w = graphgen.weights(row, col, 64)
    n = row.size - 1
    g = _load(ctx, row, col, w)
    src = graphgen.sample_sources(row, col, 64)
    _say("host outputs rmat18 k=64")
    dev = ctx.sssp_batch(g, src).cpu().numpy().view(np.uint32)
    host = np.empty(64 * n, np.uint32)
    ctx.sssp_batch(g, src, out=host)
    assert np.array_equal(host, dev)
    pinned = torch.empty(64 * n, dtype=torch.int32, pin_memory=True)
    ctx.bfs_batch(g, src, out=pinned)
    assert np.array_equal(pinned.numpy(), ctx.bfs_batch(g, src).cpu().numpy())
    assert np.array_equal(pinned.numpy()[:n], oracle.bfs(row, col, src[0]))
    g.free()


@pytest.mark.parametrize("alpha", [1, 2, 4, 8, 16, 64])
def test_bfs_batch_every_switch_point_rmat20(ctx, alpha):
    """MS-BFS at each push->pull switch point the autotuner tries, on a graph
    large enough for the switch to fall between several levels."""
    row, col = _rmat20()
    n = row.size - 1
    deg = np.diff(row)
    rng = np.random.default_rng(7)
    src = np.concatenate([[int(np.argmax(deg))], rng.choice(np.nonzero(deg > 0)[0], 63, replace=False)]).astype(np.int32)
    g = _load(ctx, row, col)
    ctx.set_option("msbfs.alpha", alpha)
    ctx.set_option("batch.min_bfs", 1)
    try:
        _say("bfs_batch rmat20 alpha", alpha)
        d = _host(ctx.bfs_batch(g, src)).reshape(64, n)
        for i in (0, 1, 17, 40, 63):
            assert np.array_equal(d[i], oracle.bfs(row, col, src[i])), (alpha, i)
    finally:
        ctx.set_option("msbfs.alpha", 4)
        ctx.set_option("batch.min_bfs", 8)
        g.free()


_R20 = {}


def _rmat20():
    if not _R20:
        _R20["g"] = graphgen.rmat(20)
    return _R20["g"]


def test_output_reuse_is_ordered_with_the_default_stream(ctx):
    """A copy of an output taken on PyTorch's default stream, immediately
    followed by another call into the same buffer, sees the first result: the
    call's work is ordered after work queued on the default stream."""
    import torch
    row, col = _rmat20()
    n = row.size - 1
    g = _load(ctx, row, col)
    src = graphgen.sample_sources(row, col, 64)
    buf = torch.empty(64 * n, dtype=torch.int32, device="cuda")
    _say("output reuse rmat20")
    ctx.set_option("batch.min_bfs", 1)
    try:
        copies = []
        for _ in range(3):
            ctx.bfs_batch(g, src, out=buf)
            copies.append(buf.clone())          # queued on the default stream, not waited for
        for c in copies:
            h = c.cpu().numpy().reshape(64, n)
            for i in (0, 31, 63):
                assert np.array_equal(h[i], oracle.bfs(row, col, src[i])), i
    finally:
        ctx.set_option("batch.min_bfs", 8)
        g.free()


@pytest.mark.parametrize("name", ["rmat16", "grid96", "star5000", "forest"])
@pytest.mark.parametrize("alpha", [0.5, 1e6])
def test_sssp_batch_pull_sweeps(ctx, name, alpha):
    """Batched SSSP with pull sweeps (alpha 1e6: every iteration pulls; 0.5:
    only frontiers carrying more than twice the edges, i.e. none after the
    first few) equals the oracle; duplicated and isolated sources included."""
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(3)
    src = rng.integers(0, n, size=40).astype(np.int32)
    src[1] = src[2]
    iso = np.nonzero(np.diff(row) == 0)[0]
    if iso.size:
        src[-1] = iso[0]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.pull_alpha", alpha)
    ctx.set_option("batch.min_sssp", 1)
    try:
        _say("sssp_batch pull", name, alpha)
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, n)
        if alpha > 1:
            assert ctx.stat("pull_iterations") > 0
        for i in (0, 1, 2, 17, src.size - 1):
            assert np.array_equal(s[i], oracle.sssp(row, col, w, src[i])), (name, alpha, i)
    finally:
        ctx.set_option("batch.pull_alpha", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("name", ["rmat16", "grid96", "path3000", "star5000"])
@pytest.mark.parametrize("narrow", [0, 2, 3])
def test_sssp_batch_row_width(ctx, name, narrow):
    """Batched SSSP with 32-bit distance rows (narrow 0), with 16-bit rows
    tried first (narrow 2) and with 8-bit rows tried first (narrow 3) equals
    the oracle.  Where distances outgrow a width (the lattice's weights go up
    to 1000, the long path), the attempt overflows and the batch is solved
    again with rows twice as wide.  A tentative distance may outgrow a width
    that the final ones fit, so a fallback is allowed there, never a narrower
    finish than the final distances fit."""
    row, col, w = graph(name)
    n = row.size - 1
    rng = np.random.default_rng(5)
    src = rng.integers(0, n, size=70).astype(np.int32)   # two batches, the second ragged
    src[0] = 0
    src[1] = src[2]
    g = _load(ctx, row, col, w)
    ctx.set_option("batch.narrow", narrow)
    ctx.set_option("batch.min_sssp", 1)
    try:
        _say("sssp_batch row width", name, narrow)
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, n)
        b8, b16, fb = ctx.stat("batches_8bit"), ctx.stat("batches_16bit"), ctx.stat("narrow_fallbacks")
        ref = [oracle.sssp(row, col, w, int(x)) for x in src]
        for i in range(src.size):
            assert np.array_equal(s[i], ref[i]), (name, narrow, i)
        maxd = max(int(r[r != 0xFFFFFFFF].max()) for r in ref)
        _say("max distance", maxd, "8-bit batches", b8, "16-bit batches", b16, "fallbacks", fb)
        if narrow == 0:
            assert b8 == 0 and b16 == 0 and fb == 0
        elif narrow == 2:
            assert b8 == 0
            if maxd >= 0xFFFF:
                assert b16 == 0 and fb >= 1
        else:
            if maxd >= 0xFF:
                assert b8 == 0 and fb >= 1
            if maxd >= 0xFFFF:
                assert b16 == 0 and fb >= 2
        if narrow and maxd < 0xFF and name == "star5000":
            # one path per vertex: tentative distances are final ones
            assert fb == 0 and (b8 if narrow == 3 else b16) == 2
    finally:
        ctx.set_option("batch.narrow", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("second", [0x7F, 0x80, 0xFE])
def test_sssp_batch_8bit_boundary(ctx, second):
    """Path 0 - 1 - 2 with weights 0x7F and `second`: the far end sits at 0xFE
    (the largest 8-bit distance), at 0xFF (does not fit: solved again with
    16-bit rows) or at 0x17D; four queries share each 32-bit word of a row,
    and every result equals the oracle."""
    row = np.array([0, 1, 3, 4], np.int32)
    col = np.array([1, 0, 2, 1], np.int32)
    w = np.array([0x7F, 0x7F, second, second], np.uint32)
    g = _load(ctx, row, col, w)
    src = np.array([0, 2, 1, 0, 2, 2, 1, 0], np.int32)
    ctx.set_option("batch.narrow", 3)
    ctx.set_option("batch.min_sssp", 1)
    try:
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, 3)
        for i in range(src.size):
            assert np.array_equal(s[i], oracle.sssp(row, col, w, int(src[i]))), (second, i)
        fits = 0x7F + second < 0xFF
        assert ctx.stat("batches_8bit") == (1 if fits else 0)
        assert ctx.stat("batches_16bit") == (0 if fits else 1)
        assert ctx.stat("narrow_fallbacks") == (0 if fits else 1)
    finally:
        ctx.set_option("batch.narrow", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()


@pytest.mark.parametrize("second", [0x7FFF, 0x8000, 0xFFFE])
def test_sssp_batch_narrow_boundary(ctx, second):
    """Path 0 - 1 - 2 with weights 0x7FFF and `second`: the far end sits at
    0xFFFE (the largest narrow distance), at 0xFFFF (does not fit: solved
    again with wide rows) or at 0x17FFD; every result equals the oracle."""
    row = np.array([0, 1, 3, 4], np.int32)
    col = np.array([1, 0, 2, 1], np.int32)
    w = np.array([0x7FFF, 0x7FFF, second, second], np.uint32)
    g = _load(ctx, row, col, w)
    src = np.array([0, 2, 1, 0], np.int32)
    ctx.set_option("batch.narrow", 2)
    ctx.set_option("batch.min_sssp", 1)
    try:
        s = _host(ctx.sssp_batch(g, src)).view(np.uint32).reshape(src.size, 3)
        for i in range(src.size):
            assert np.array_equal(s[i], oracle.sssp(row, col, w, int(src[i]))), (second, i)
        fits = 0x7FFF + second < 0xFFFF
        assert ctx.stat("narrow_batches") == (1 if fits else 0)
        assert ctx.stat("narrow_fallbacks") == (0 if fits else 1)
    finally:
        ctx.set_option("batch.narrow", 0)
        ctx.set_option("batch.min_sssp", 24)
        g.free()
