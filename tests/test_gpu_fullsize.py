"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the bench times (the packaged tuning file, 64-source batches),
on outputs the oracle computes one by one, plus properties that hold at any
size for every output the oracle does not recompute:

* R-MAT s22, 64 sources, BFS + SSSP (the bench step): three rows of each
  against the oracle; every row of both checked by the BFS and shortest-path
  invariants over all 128 M directed edges.
* 4096^2 perturbed lattice with long edges (16.8 M vertices): BFS, SSSP and
  CC against the oracle.
* R-MAT s23: BC from 4 sources against the oracle; BC from 32 sources
  against the identity sum_v BC(v) = sum_s sum_t (d(s,t) - 1); PageRank
  against the FP64 oracle run for the GPU's iteration count; filtered
  PageRank against the oracle of the same method (iterations and final
  frontier exact).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_05387_amd as gfr
    c = gfr.Context(0, tuning_json=gfr.tuned_json())
    yield c
    c.close()


def _edges(row, col, dev):
    import torch
    R = torch.from_numpy(row.astype(np.int64)).to(dev)
    src = torch.repeat_interleave(torch.arange(row.size - 1, device=dev), R[1:] - R[:-1])
    return src, torch.from_numpy(col.astype(np.int64)).to(dev)


def test_rmat22_bench_step(ctx):
    import torch
    dev = torch.device("cuda:0")
    row, col = graphgen.rmat(22)
    w = graphgen.weights(row, col, 64)
    n = row.size - 1
    srcs = graphgen.sample_sources(row, col, 64)
    g = ctx.graph_load_csr(row, col, w)
    _say("rmat22 bfs_batch + sssp_batch, 64 sources")
    dep = ctx.bfs_batch(g, srcs).view(64, n)
    dist = ctx.sssp_batch(g, srcs).view(64, n)
    for i in (0, 31, 63):
        assert np.array_equal(dep[i].cpu().numpy(), oracle.bfs(row, col, srcs[i])), i
        assert np.array_equal(dist[i].cpu().numpy().view(np.uint32), oracle.sssp(row, col, w, srcs[i])), i
    # every row: invariants over all directed edges
    eu, ev = _edges(row, col, dev)
    W = torch.from_numpy(w.astype(np.int64)).to(dev)
    for i in range(64):
        d = dep[i].to(torch.int64)
        assert d[int(srcs[i])] == 0
        du, dv = d[eu], d[ev]
        assert bool(((du >= 0) == (dv >= 0)).all()), ("reached set not closed", i)
        both = du >= 0
        assert bool(((du - dv).abs()[both] <= 1).all()), ("BFS edge rule", i)
        s = dist[i].to(torch.int64) & 0xFFFFFFFF
        su, sv = s[eu], s[ev]
        fin = su != 0xFFFFFFFF
        assert bool((fin == (sv != 0xFFFFFFFF)).all()), ("SSSP reach", i)
        assert bool((sv[fin] <= su[fin] + W[fin]).all()), ("triangle inequality", i)
        assert bool((fin == both).all()), ("SSSP and BFS reach differ", i)
        # every reached vertex but the source has a tight in-edge
        tight = torch.zeros(n, dtype=torch.bool, device=dev)
        tight[ev[fin & (su + W == sv)]] = True
        reached = s != 0xFFFFFFFF
        reached[int(srcs[i])] = False
        assert bool(tight[reached].all()), ("tight edge", i)
    g.free()


def test_rmat22_predecessors(ctx):
    row, col = graphgen.rmat(22)
    w = graphgen.weights(row, col, 64)
    src = int(graphgen.sample_sources(row, col, 1)[0])
    g = ctx.graph_load_csr(row, col, w)
    _say("rmat22 bfs/sssp predecessors from", src)
    d, p = ctx.bfs(g, src, pred=True)
    do, po = oracle.bfs_pred(row, col, src)
    assert np.array_equal(d.cpu().numpy(), do) and np.array_equal(p.cpu().numpy(), po)
    d, p = ctx.sssp(g, src, pred=True)
    do, po = oracle.sssp_pred(row, col, w, src)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), do) and np.array_equal(p.cpu().numpy(), po)
    g.free()


def test_grid4096_bfs_sssp_cc(ctx):
    row, col = graphgen.grid(4096)
    w = graphgen.weights(row, col, 1000)
    src = int(graphgen.sample_sources(row, col, 1)[0])
    g = ctx.graph_load_csr(row, col, w)
    _say("grid4096 bfs/sssp/cc from", src)
    assert np.array_equal(ctx.bfs(g, src).cpu().numpy(), oracle.bfs(row, col, src))
    assert np.array_equal(ctx.sssp(g, src).cpu().numpy().view(np.uint32), oracle.sssp(row, col, w, src))
    lab, k = ctx.cc(g)
    ref, kref = oracle.cc(row, col)
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert k == kref
    g.free()


@pytest.fixture(scope="module")
def rmat23():
    return graphgen.rmat(23)


def test_rmat23_bc(ctx, rmat23):
    import torch
    row, col = rmat23
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    src32 = graphgen.sample_sources(row, col, 32)
    _say("rmat23 bc, 4 sources vs oracle")
    got = ctx.bc(g, src32[:4]).cpu().numpy().astype(np.float64)
    ref = oracle.bc(row, col, src32[:4])
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)) <= 1e-5
    _say("rmat23 bc, 32 sources vs the path-length identity")
    bc32 = ctx.bc(g, src32).to(torch.float64)
    d = ctx.bfs_batch(g, src32).view(32, n).to(torch.float64)
    for i in (0, 17):
        assert np.array_equal(d[i].cpu().numpy().astype(np.int32), oracle.bfs(row, col, src32[i]))
    want = float(torch.where(d > 0, d - 1.0, torch.zeros_like(d)).sum())
    assert abs(float(bc32.sum()) - want) <= 1e-5 * want
    assert float(bc32.min()) >= 0.0
    g.free()


def test_rmat23_pagerank(ctx, rmat23):
    row, col = rmat23
    g = ctx.graph_load_csr(row, col)
    _say("rmat23 pagerank")
    rank, it, l1 = ctx.pagerank(g, 0.85, 1e-6, 1000)
    ref, it_ref, _ = oracle.pagerank(row, col, 0.85, 0.0, it)
    assert it_ref == it
    err = float(np.abs(rank.cpu().numpy().astype(np.float64) - ref).sum())
    _say("rmat23 pagerank iterations", it, "L1 vs FP64 oracle", err)
    assert err <= 1e-6
    assert abs(float(rank.sum()) - 1.0) <= 1e-5
    g.free()


def test_rmat23_pagerank_filtered(ctx, rmat23):
    row, col = rmat23
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    eps = 1e-4 / n
    _say("rmat23 pagerank_filtered, vertex_tol 1e-4/N")
    x, act, it, l1 = ctx.pagerank_filtered(g, 0.85, eps, 1000)
    xo, ito, l1o, acto = oracle.pagerank_filtered(row, col, 0.85, eps, 1000)
    assert it == ito
    assert np.array_equal(act.cpu().numpy().astype(bool), acto)
    err = float(np.abs(x.cpu().numpy() - xo).sum())
    _say("rmat23 pagerank_filtered iterations", it, "L1 vs oracle", err)
    assert err <= 1e-11
    assert abs(l1 - l1o) <= 1e-12 + 1e-9 * l1o
    g.free()
