"""The BFS entry point that allocates nothing (gfr_bfs_noalloc) against the
ordinary one (gfr_bfs) and the oracle, through the C ABI.

Two calls in a row on one context, the second on a smaller graph (so the
fixed scratch still holds the first call's larger state), on a scale-free
graph (queue levels, per-level push/pull) and on a lattice (mark-byte
levels); plus the errors: a host output, a source out of range, and a graph
whose traversal needs more scratch than the fixed array holds.
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


def _both(ctx, row, col, src):
    import torch
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    out = torch.full((n,), 7, dtype=torch.int32, device="cuda:0")
    got = ctx.bfs_noalloc(g, src, out).cpu().numpy()
    ref = ctx.bfs(g, src).cpu().numpy()
    g.free()
    return got, ref


@pytest.mark.parametrize("kind", ["rmat", "grid"])
def test_noalloc_matches_bfs_twice_second_smaller(ctx, kind):
    if kind == "rmat":
        graphs = [graphgen.rmat(16), graphgen.rmat(11)]
    else:
        graphs = [graphgen.grid(160), graphgen.grid(40)]
    for call, (row, col) in enumerate(graphs):
        src = int(graphgen.sample_sources(row, col, 1, seed=11 + call)[0])
        _say("bfs_noalloc", kind, "call", call, "n", row.size - 1, "source", src)
        got, ref = _both(ctx, row, col, src)
        assert np.array_equal(got, ref), (kind, call)
        assert np.array_equal(got, oracle.bfs(row, col, src)), (kind, call)


def test_noalloc_rejects_host_output_and_bad_source(ctx):
    import paper_1501_05387_amd as gfr
    import torch
    row, col = graphgen.rmat(10)
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    host = np.zeros(n, np.int32)
    with pytest.raises(gfr.GfrError) as e:
        ctx.bfs_noalloc(g, 0, host)
    assert e.value.status == -1
    dev = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gfr.GfrError) as e:
        ctx.bfs_noalloc(g, n, dev)
    assert e.value.status == -1
    g.free()


def test_noalloc_rejects_a_graph_beyond_the_scratch(ctx):
    import paper_1501_05387_amd as gfr
    import torch
    # a path of 6 M vertices needs about 13.25 B per vertex = 79 MB of scratch > 64 MiB
    n = 6_000_000
    row, col = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    g = ctx.graph_load_csr(row, col)
    ctx.set_option("bfs.frontier", 1)   # the queue form (the lattice-class default needs only 2 B per vertex)
    try:
        out = torch.full((n,), 5, dtype=torch.int32, device="cuda:0")
        _say("bfs_noalloc capacity check, n", n)
        with pytest.raises(gfr.GfrError) as e:
            ctx.bfs_noalloc(g, 0, out)
        assert e.value.status == -6
        assert "scratch" in str(e.value)
        assert bool((out == 5).all()), "a rejected call wrote its output"
    finally:
        ctx.set_option("bfs.frontier", 0)
        g.free()
