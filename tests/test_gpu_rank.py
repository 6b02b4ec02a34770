"""GPU parity for the 2-hop advance and the node rankings (personalized
PageRank, SALSA, HITS) against the CPU oracle, through the C ABI.

2-hop walk counts are integers and must match bit for bit, in both
directions of the second advance; the FP64 rankings must agree within 1e-12
(absolute, per score), PPR at the GPU's own iteration count.
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


def _star(k):
    return graphgen.from_edges(k + 1, np.zeros(k, np.int32), np.arange(1, k + 1))


GRAPHS = {
    "rmat12": lambda: graphgen.rmat(12),
    "rmat16": lambda: graphgen.rmat(16),
    "grid96": lambda: graphgen.grid(96),
    "star5000": lambda: _star(5000),
    "forest": lambda: graphgen.from_edges(2000, np.arange(0, 1998, 2), np.arange(1, 1999, 2)),
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def _seeds(row, k, seed=11):
    n = row.size - 1
    rng = np.random.default_rng(seed)
    s = rng.choice(n, size=min(k, n), replace=False)
    s[0] = 0                                   # the top hub of an R-MAT graph, the star's centre
    return np.unique(s).astype(np.int32)


# ----------------------------------------------------------------- 2-hop
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("k", [1, 7, 64])
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_two_hop_matches_oracle(ctx, name, k, direction):
    row, col = graph(name)
    S = _seeds(row, k)
    g = ctx.graph_load_csr(row, col)
    _say("two_hop", name, "k", S.size, "direction", direction)
    ctx.set_option("twohop.direction", direction)
    try:
        got = _host(ctx.two_hop(g, S)).view(np.uint64)
    finally:
        ctx.set_option("twohop.direction", 0)
    assert np.array_equal(got, oracle.two_hop(row, col, S))
    g.free()


def test_two_hop_host_output_and_edge_cases(ctx):
    import paper_1501_05387_amd as gfr
    row, col = graph("rmat12")
    g = ctx.graph_load_csr(row, col)
    out = np.empty(row.size - 1, np.uint64)
    S = _seeds(row, 9)
    assert ctx.two_hop(g, S, out=out) is out
    assert np.array_equal(out, oracle.two_hop(row, col, S))
    iso = int(np.nonzero(np.diff(row) == 0)[0][0])
    assert not _host(ctx.two_hop(g, [iso])).any()
    for bad in ([], [1, 1], [row.size - 1], [-1]):
        with pytest.raises(gfr.GfrError) as ei:
            ctx.two_hop(g, bad)
        assert ei.value.status == gfr.GFR_E_INVALID
    g.free()
    g = ctx.graph_load_csr(np.zeros(6, np.int32), np.zeros(0, np.int32))
    assert not _host(ctx.two_hop(g, [0, 3])).any()
    g.free()


# ------------------------------------------------------------------- PPR
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("k", [1, 16])
def test_ppr_matches_oracle(ctx, name, k):
    row, col = graph(name)
    S = _seeds(row, k, seed=12)
    g = ctx.graph_load_csr(row, col)
    _say("ppr", name, "k", S.size)
    x, it, l1 = ctx.ppr(g, S, 0.85, 1e-10, 1000)
    x = _host(x)
    xo, ito, l1o = oracle.ppr(row, col, S, 0.85, 0.0, it)
    assert ito == it
    err = float(np.abs(x - xo).sum())
    _say("ppr", name, "iterations", it, "L1 vs oracle", err)
    assert err <= 1e-12
    assert abs(l1 - l1o) <= 1e-12
    _, it_ref, _ = oracle.ppr(row, col, S, 0.85, 1e-10, 1000)
    assert abs(it - it_ref) <= 1
    g.free()


def test_ppr_host_output_and_edge_cases(ctx):
    import paper_1501_05387_amd as gfr
    row, col = graph("star5000")
    g = ctx.graph_load_csr(row, col)
    out = np.empty(row.size - 1, np.float64)
    x, it, _ = ctx.ppr(g, [3, 0], 0.5, 0.0, 12, out=out)
    assert x is out and it == 12
    assert np.abs(out - oracle.ppr(row, col, [3, 0], 0.5, 0.0, 12)[0]).sum() <= 1e-12
    for call in (lambda: ctx.ppr(g, [1, 1]), lambda: ctx.ppr(g, [0], 1.0), lambda: ctx.ppr(g, [0], 0.85, -1.0),
                 lambda: ctx.ppr(g, [0], 0.85, 1e-9, 0)):
        with pytest.raises(gfr.GfrError) as ei:
            call()
        assert ei.value.status == gfr.GFR_E_INVALID
    g.free()
    row = np.zeros(6, np.int32)
    g = ctx.graph_load_csr(row, np.zeros(0, np.int32))
    x, it, l1 = ctx.ppr(g, [1, 4], 0.85, 1e-9, 100)
    xo, ito, _ = oracle.ppr(row, np.zeros(0, np.int32), [1, 4], 0.85, 1e-9, 100)
    assert it == ito and np.abs(_host(x) - xo).sum() <= 1e-15
    g.free()


# ---------------------------------------------------------- SALSA / HITS
def _bip_random(nl, nr, p, seed):
    rng = np.random.default_rng(seed)
    l, r = np.nonzero(rng.random((nl, nr)) < p)
    return graphgen.from_edges(nl + nr, l, nl + r), nl


BIP = {
    "bip_rmat10": lambda: (graphgen.bipartite_rmat(10), 1 << 10),
    "bip_rmat15": lambda: (graphgen.bipartite_rmat(15), 1 << 15),
    "random_with_isolated": lambda: _bip_random(300, 700, 0.004, 3),
    "k_3_5": lambda: (graphgen.from_edges(8, np.repeat(np.arange(3), 5), 3 + np.tile(np.arange(5), 3)), 3),
}


@pytest.mark.parametrize("name", list(BIP))
@pytest.mark.parametrize("iters", [0, 1, 5, 30])
@pytest.mark.parametrize("method", ["salsa", "hits"])
def test_bipartite_rank_matches_oracle(ctx, name, iters, method):
    (row, col), nl = BIP[name]()
    g = ctx.graph_load_csr(row, col)
    _say(method, name, "iters", iters)
    h, a = getattr(ctx, method)(g, nl, iters)
    ho, ao = getattr(oracle, method)(row, col, nl, iters)
    h, a = _host(h), _host(a)
    assert h.shape == ho.shape and a.shape == ao.shape
    assert np.max(np.abs(h - ho)) <= 1e-12 and np.max(np.abs(a - ao)) <= 1e-12
    g.free()


def test_bipartite_host_outputs_and_checks(ctx):
    import paper_1501_05387_amd as gfr
    (row, col), nl = BIP["bip_rmat10"]()
    g = ctx.graph_load_csr(row, col)
    hub, auth = np.empty(nl), np.empty(row.size - 1 - nl)
    h, a = ctx.salsa(g, nl, 7, hub=hub, auth=auth)
    assert h is hub and a is auth
    ho, ao = oracle.salsa(row, col, nl, 7)
    assert np.max(np.abs(hub - ho)) <= 1e-12 and np.max(np.abs(auth - ao)) <= 1e-12
    assert row[nl + 1] > row[nl]
    for bad_nl in (0, row.size - 1, nl + 1):     # nl + 1 moves a right vertex with edges to the left
        with pytest.raises(gfr.GfrError) as ei:
            ctx.hits(g, bad_nl, 3)
        assert ei.value.status == gfr.GFR_E_INVALID
    h, a = ctx.hits(g, nl, 3)                    # the failed checks leave the graph usable
    assert np.max(np.abs(_host(h) - oracle.hits(row, col, nl, 3)[0])) <= 1e-12
    g.free()


def test_rankings_on_a_graph_without_edges(ctx):
    row = np.zeros(8, np.int32)
    col = np.zeros(0, np.int32)
    g = ctx.graph_load_csr(row, col)
    for method in ("salsa", "hits"):
        for iters in (0, 1, 3):
            h, a = getattr(ctx, method)(g, 3, iters)
            ho, ao = getattr(oracle, method)(row, col, 3, iters)
            assert np.array_equal(_host(h), ho) and np.array_equal(_host(a), ao), (method, iters)
    assert not _host(ctx.two_hop(g, [0, 6])).any()
    g.free()
