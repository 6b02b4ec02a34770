"""GPU parity for the advance and filter operators on their own, through the
C ABI, against their definitions: every frontier edge exactly once, in
frontier order then CSR order (from a vertex or from an edge frontier);
filter = the ascending distinct kept ids; scan = the exact exclusive prefix
sum; split = the near and far lists in input order.
The graphs include a hub spanning several load-balancing chunks and rows
whose degrees sit at the wave and chunk sizes and one either side."""
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


def _cutoffs():
    """Hubs of degree 63, 64, 65, 1023, 1024, 1025 and 2049, each on leaves of its own."""
    eu, ev, nxt = [], [], 7
    for h, d in enumerate((63, 64, 65, 1023, 1024, 1025, 2049)):
        eu += [h] * d
        ev += list(range(nxt, nxt + d))
        nxt += d
    return graphgen.from_edges(nxt + 5, eu, ev)      # five isolated vertices at the end


GRAPHS = {
    "rmat12": lambda: graphgen.rmat(12),
    "rmat16": lambda: graphgen.rmat(16),
    "grid96": lambda: graphgen.grid(96),
    "star5000": lambda: graphgen.from_edges(5001, np.zeros(5000, np.int32), np.arange(1, 5001)),
    "cutoffs": _cutoffs,
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def _frontiers(row, seed=5):
    n = row.size - 1
    rng = np.random.default_rng(seed)
    deg = np.diff(row)
    iso = np.nonzero(deg == 0)[0]
    out = {
        "empty": np.zeros(0, np.int32),
        "one": np.array([0], np.int32),
        "random_dup_100": rng.integers(0, n, size=100).astype(np.int32),
        "random_dup_5000": rng.integers(0, n, size=5000).astype(np.int32),
        "all_reversed": np.arange(n - 1, -1, -1, dtype=np.int32),
    }
    if iso.size:
        out["isolated_only"] = np.repeat(iso[:3], 2).astype(np.int32)
    return out


@pytest.mark.parametrize("name", list(GRAPHS))
def test_advance_matches_definition(ctx, name):
    import torch
    row, col = graph(name)
    g = ctx.graph_load_csr(row, col)
    for fname, F in _frontiers(row).items():
        _say("advance", name, fname, F.size)
        src, edge, dst = oracle.advance(row, col, F)
        for inp in (F, torch.from_numpy(F).cuda()):     # host and device frontiers
            s, e, d = ctx.advance(g, inp)
            assert np.array_equal(s.cpu().numpy(), src)
            assert np.array_equal(e.cpu().numpy(), edge)
            assert np.array_equal(d.cpu().numpy(), dst)
    g.free()


def test_advance_capacity_and_errors(ctx):
    import ctypes
    import paper_1501_05387_amd as gfr
    row, col = graph("cutoffs")
    g = ctx.graph_load_csr(row, col)
    F = np.arange(7, dtype=np.int32)
    total = int(np.diff(row)[:7].sum())
    with pytest.raises(gfr.GfrError) as ei:
        ctx.advance(g, F, out_cap=total - 1)
    assert ei.value.status == gfr.GFR_E_CAPACITY
    cnt = ctypes.c_int64()
    st = gfr.lib().gfr_advance(ctx.ptr, g.handle, F.ctypes.data, F.size, None, None, None, 0, ctypes.byref(cnt), None)
    assert st == gfr.GFR_E_CAPACITY and cnt.value == total
    s, e, d = ctx.advance(g, F, out_cap=total)
    assert s.numel() == total
    for bad in ([row.size - 1], [-1]):
        with pytest.raises(gfr.GfrError) as ei:
            ctx.advance(g, np.array(bad, np.int32))
        assert ei.value.status == gfr.GFR_E_INVALID
    out = np.empty(total, np.int32)                      # host outputs are refused
    st = gfr.lib().gfr_advance(ctx.ptr, g.handle, F.ctypes.data, F.size, out.ctypes.data, None, None, total,
                               ctypes.byref(cnt), None)
    assert st == gfr.GFR_E_INVALID
    g.free()


def _edge_frontiers(row, col, seed=7):
    m = col.size
    rng = np.random.default_rng(seed)
    deg = np.diff(row)
    into_big = np.nonzero(deg[col] >= 63)[0]        # edges whose far end spans one or more chunks
    out = {
        "empty": np.zeros(0, np.int32),
        "one": np.array([0], np.int32),
        "last": np.array([m - 1], np.int32),
        "random_dup_100": rng.integers(0, m, size=100).astype(np.int32),
        "random_dup_5000": rng.integers(0, m, size=5000).astype(np.int32),
        "into_big_dup": np.repeat(into_big[:40], 2).astype(np.int32),
    }
    if int((deg.astype(np.int64) ** 2).sum()) <= 20_000_000:
        out["all_edges_reversed"] = np.arange(m - 1, -1, -1, dtype=np.int32)
    return out


@pytest.mark.parametrize("name", list(GRAPHS))
def test_edge_advance_matches_definition(ctx, name):
    import torch
    row, col = graph(name)
    g = ctx.graph_load_csr(row, col)
    for fname, E in _edge_frontiers(row, col).items():
        _say("advance_edges", name, fname, E.size)
        src, edge, dst = oracle.advance_edges(row, col, E)
        for inp in (E, torch.from_numpy(E).cuda()):     # host and device frontiers
            s, e, d = ctx.advance_edges(g, inp)
            assert np.array_equal(s.cpu().numpy(), src)
            assert np.array_equal(e.cpu().numpy(), edge)
            assert np.array_equal(d.cpu().numpy(), dst)
    g.free()


def test_edge_advance_capacity_and_errors(ctx):
    import ctypes
    import paper_1501_05387_amd as gfr
    row, col = graph("cutoffs")
    g = ctx.graph_load_csr(row, col)
    into_hub = np.nonzero(col < 7)[0]
    E = np.array([into_hub[0], into_hub[-1], col.size - 1], np.int32)   # into hubs 0 and 6, and the last edge
    deg = np.diff(row)
    total = int(deg[col[E]].sum())
    with pytest.raises(gfr.GfrError) as ei:
        ctx.advance_edges(g, E, out_cap=total - 1)
    assert ei.value.status == gfr.GFR_E_CAPACITY
    cnt = ctypes.c_int64()
    st = gfr.lib().gfr_advance_edges(ctx.ptr, g.handle, E.ctypes.data, E.size, None, None, None, 0,
                                     ctypes.byref(cnt), None)
    assert st == gfr.GFR_E_CAPACITY and cnt.value == total
    s, e, d = ctx.advance_edges(g, E, out_cap=total)
    assert s.numel() == total
    for bad in ([col.size], [-1], [0, col.size + 5]):
        with pytest.raises(gfr.GfrError) as ei:
            ctx.advance_edges(g, np.array(bad, np.int32))
        assert ei.value.status == gfr.GFR_E_INVALID
    g.free()


@pytest.mark.parametrize("name", list(GRAPHS))
def test_filter_matches_definition(ctx, name):
    import torch
    row, col = graph(name)
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    rng = np.random.default_rng(6)
    ex = (rng.random(n) < 0.3).astype(np.uint8)
    for fname, X in _frontiers(row).items():
        _say("filter", name, fname, X.size)
        assert np.array_equal(ctx.filter(g, X).cpu().numpy(), oracle.filter_ids(n, X))
        want = oracle.filter_ids(n, X, ex)
        assert np.array_equal(ctx.filter(g, X, ex).cpu().numpy(), want)
        got = ctx.filter(g, torch.from_numpy(X).cuda(), torch.from_numpy(ex).cuda())
        assert np.array_equal(got.cpu().numpy(), want)
    assert ctx.filter(g, np.arange(n, dtype=np.int32), np.ones(n, np.uint8)).numel() == 0
    g.free()


SCAN_SIZES = (0, 1, 2047, 2048, 2049, 100_000, 3_000_001)   # tile is 2048: empty, one, ragged, several tiles


@pytest.mark.parametrize("count", SCAN_SIZES)
def test_scan_matches_definition(ctx, count):
    import torch
    rng = np.random.default_rng(count + 1)
    for kind in ("small", "full"):
        hi = 100 if kind == "small" else 2**32
        v = rng.integers(0, hi, size=count, dtype=np.uint64).astype(np.uint32)
        _say("scan", count, kind)
        want, tot = oracle.scan(v)
        for inp in (v, torch.from_numpy(v.view(np.int32)).cuda()):   # host and device input
            out, total = ctx.scan(inp)
            assert total == tot
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want)


def test_scan_past_2_pow_53(ctx):
    v = np.full(3_000_000, 2**32 - 1, np.uint32)
    out, total = ctx.scan(v)
    assert total == 3_000_000 * (2**32 - 1)
    got = out.cpu().numpy().view(np.uint64)
    assert int(got[-1]) == 2_999_999 * (2**32 - 1) and int(got[1_234_567]) == 1_234_567 * (2**32 - 1)


@pytest.mark.parametrize("name", ["rmat12", "grid96", "cutoffs"])
def test_split_matches_definition(ctx, name):
    import torch
    row, col = graph(name)
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    rng = np.random.default_rng(13)
    dist = rng.integers(0, 1000, size=n, dtype=np.uint64).astype(np.uint32)
    dist[:5] = 0xFFFFFFFF                                          # unreached vertices are always far
    for fname, X in _frontiers(row).items():
        for thr in (0, 1, 500, 1000, 0xFFFFFFFF):
            _say("split", name, fname, X.size, thr)
            near, far = oracle.split(X, dist, thr)
            for xs, ds in ((X, dist), (torch.from_numpy(X).cuda(), torch.from_numpy(dist.view(np.int32)).cuda())):
                gn, gf = ctx.split(g, xs, ds, thr)
                assert np.array_equal(gn.cpu().numpy(), near)
                assert np.array_equal(gf.cpu().numpy(), far)
    g.free()


def test_split_capacity_and_errors(ctx):
    import ctypes
    import paper_1501_05387_amd as gfr
    row, col = graph("grid96")
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    dist = (np.arange(n) % 7).astype(np.uint32)
    X = np.arange(100, dtype=np.int32)
    want_near, want_far = oracle.split(X, dist, 3)
    nn, nf = ctypes.c_int64(), ctypes.c_int64()
    st = gfr.lib().gfr_split(ctx.ptr, g.handle, X.ctypes.data, X.size, dist.ctypes.data, 3, None, None, 0,
                             ctypes.byref(nn), ctypes.byref(nf), None)
    assert st == gfr.GFR_E_CAPACITY and (nn.value, nf.value) == (want_near.size, want_far.size)
    for bad in ([n], [-1]):
        with pytest.raises(gfr.GfrError) as ei:
            ctx.split(g, np.array(bad, np.int32), dist, 3)
        assert ei.value.status == gfr.GFR_E_INVALID
    out = np.empty(100, np.int32)                                  # host outputs are refused
    st = gfr.lib().gfr_split(ctx.ptr, g.handle, X.ctypes.data, X.size, dist.ctypes.data, 3, out.ctypes.data,
                             out.ctypes.data, 100, ctypes.byref(nn), ctypes.byref(nf), None)
    assert st == gfr.GFR_E_INVALID
    g.free()


def test_operators_on_a_graph_without_edges(ctx):
    import paper_1501_05387_amd as gfr
    row = np.zeros(9, np.int32)
    g = ctx.graph_load_csr(row, np.zeros(0, np.int32))
    s, e, d = ctx.advance(g, np.array([3, 3, 0], np.int32))
    assert s.numel() == 0 and e.numel() == 0 and d.numel() == 0
    assert ctx.advance_edges(g, np.zeros(0, np.int32))[0].numel() == 0
    with pytest.raises(gfr.GfrError) as ei:               # no edge id is valid
        ctx.advance_edges(g, np.array([0], np.int32))
    assert ei.value.status == gfr.GFR_E_INVALID
    assert ctx.filter(g, np.array([5, 1, 5, 7], np.int32)).cpu().numpy().tolist() == [1, 5, 7]
    g.free()
