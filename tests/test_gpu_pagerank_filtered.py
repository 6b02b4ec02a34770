"""GPU parity for PageRank with per-vertex convergence filtering (Sec. 5.5)
against the FP64 oracle of the same method, through the C ABI.

The filter decision is taken in FP64 on both sides, so the iteration count and
the final frontier membership must match exactly; ranks differ only by the
order of FP64 additions (within 1e-12 in L1).  An error report against the
exact fixed point (the oracle run to 1e-15) is printed per tolerance: the
method is an approximation, and the report shows how far each tolerance
lands from the answer and how much of the work it skips.
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


def _star_iso(k, n_iso):
    return graphgen.from_edges(1 + k + n_iso, np.zeros(k, np.int32), np.arange(1, k + 1))


GRAPHS = {
    "rmat12": lambda: graphgen.rmat(12),
    "rmat16": lambda: graphgen.rmat(16),
    "grid96": lambda: graphgen.grid(96),
    "star5000_iso7": lambda: _star_iso(5000, 7),
    "forest": lambda: graphgen.from_edges(2000, np.arange(0, 1998, 2), np.arange(1, 1999, 2)),
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def _check(ctx, g, row, col, d, eps, max_iter, host=False):
    n = row.size - 1
    if host:
        out, act_out = np.empty(n, np.float64), np.empty(n, np.uint8)
        x, act, it, l1 = ctx.pagerank_filtered(g, d, eps, max_iter, out=out, active=act_out)
        assert x is out and act is act_out
    else:
        x, act, it, l1 = ctx.pagerank_filtered(g, d, eps, max_iter)
    x, act = _host(x), _host(act).astype(bool)
    xo, ito, l1o, acto = oracle.pagerank_filtered(row, col, d, eps, max_iter)
    assert it == ito, (it, ito)
    assert np.array_equal(act, acto), int((act != acto).sum())
    err = float(np.abs(x - xo).sum())
    assert err <= 1e-12, err
    assert abs(l1 - l1o) <= 1e-12 + 1e-9 * l1o, (l1, l1o)
    return x, it


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("eps", [1e-12, 1e-9, 1e-6, 1e-3, 2.0])
def test_matches_oracle(ctx, name, eps):
    row, col = graph(name)
    g = ctx.graph_load_csr(row, col)
    _say("pagerank_filtered", name, "eps", eps)
    _check(ctx, g, row, col, 0.85, eps, 1000)
    g.free()


def test_zero_tolerance_is_power_iteration(ctx):
    row, col = graph("rmat12")
    g = ctx.graph_load_csr(row, col)
    for iters in (1, 7, 30):
        x, it = _check(ctx, g, row, col, 0.85, 0.0, iters)
        xp, itp, _ = oracle.pagerank(row, col, 0.85, 0.0, iters)
        assert it == iters == itp
        assert np.abs(x - xp).sum() <= 1e-12
    g.free()


def test_max_iter_caps_a_live_frontier(ctx):
    row, col = graph("rmat16")
    g = ctx.graph_load_csr(row, col)
    _, act, it, _ = ctx.pagerank_filtered(g, 0.85, 1e-12, 4)
    assert it == 4 and bool(_host(act).any())
    _check(ctx, g, row, col, 0.85, 1e-12, 4)
    _check(ctx, g, row, col, 0.5, 1e-9, 1000)
    g.free()


def test_host_outputs(ctx):
    row, col = graph("star5000_iso7")
    g = ctx.graph_load_csr(row, col)
    _check(ctx, g, row, col, 0.85, 1e-9, 1000, host=True)
    g.free()


def test_graph_without_edges(ctx):
    row = np.zeros(6, np.int32)
    col = np.zeros(0, np.int32)
    g = ctx.graph_load_csr(row, col)
    for eps in (0.0, 1e-12):
        _check(ctx, g, row, col, 0.85, eps, 5)
    g.free()


def test_deterministic_and_stats(ctx):
    row, col = graph("rmat16")
    g = ctx.graph_load_csr(row, col)
    a = [_host(ctx.pagerank_filtered(g, 0.85, 1e-9)[0]).copy() for _ in range(2)]
    assert np.array_equal(a[0], a[1])
    n = row.size - 1
    it = ctx.stat("iterations")
    upd = ctx.stat("vertex_updates")
    assert ctx.stat("final_frontier") == 0
    assert 0 < upd < it * n      # the filter skipped work
    assert 0 < ctx.stat("edges_gathered") <= it * col.size
    g.free()


def test_bad_arguments(ctx):
    import paper_1501_05387_amd as gfr
    row, col = graph("rmat12")
    g = ctx.graph_load_csr(row, col)
    for call in (lambda: ctx.pagerank_filtered(g, 1.0), lambda: ctx.pagerank_filtered(g, 0.85, -1e-9),
                 lambda: ctx.pagerank_filtered(g, 0.85, 1e-9, 0)):
        with pytest.raises(gfr.GfrError) as ei:
            call()
        assert ei.value.status == gfr.GFR_E_INVALID
    g.free()


def test_error_report_against_the_fixed_point(ctx):
    """L1 distance of the filtered result from the exact FP64 fixed point, and
    the share of vertex updates it runs, per tolerance (R-MAT s16)."""
    row, col = graph("rmat16")
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    xs, its, _ = oracle.pagerank(row, col, 0.85, 1e-15, 10000)
    prev = np.inf
    for eps in (1e-6, 1e-8, 1e-10, 1e-12):
        x, it = _check(ctx, g, row, col, 0.85, eps, 10000)
        err = float(np.abs(x - xs).sum())
        share = ctx.stat("vertex_updates") / (it * n)
        _say("eps %.0e: %d iterations, L1 error vs fixed point %.3e, vertex updates %.1f%% of %d full sweeps"
             % (eps, it, err, 100 * share, it))
        assert err < prev
        prev = err
    assert prev < 1e-6
    g.free()
