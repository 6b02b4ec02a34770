"""The autotuner and per-class tuning files on the GPU: a quick sweep over a
scale-free and a mesh graph finishes, only writes options the library accepts,
and a context built from its output still matches the oracle; per-class values
reach only graphs of their class, and explicit options beat the file."""
from __future__ import annotations

import json
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _graphs():
    r_row, r_col = graphgen.rmat(12)
    g_row, g_col = graphgen.grid(64)
    return {
        "scalefree": [("rmat12", r_row, r_col, graphgen.weights(r_row, r_col, 64))],
        "mesh": [("grid64", g_row, g_col, graphgen.weights(g_row, g_col, 1000))],
    }


def test_quick_sweep_is_results_neutral():
    import paper_1501_05387_amd as gfr
    from paper_1501_05387_amd import autotune
    graphs = _graphs()
    _say("autotune quick sweep rmat12 + grid64")
    with gfr.Context(0) as ctx:
        res = autotune.tune(ctx, graphs, quick=True, repeats=1, sources=8)
        assert set(res) == {"scalefree", "mesh"}
        for cls, opts in res.items():
            assert set(opts) == set(autotune.DEFAULTS), cls
        # the sweep restores the context's own options
        assert ctx.get_option("advance.chunk") == 1024
        assert ctx.get_option("batch.min_bfs") == 8
    text = json.dumps(res)
    _say("tuned context", text)
    with gfr.Context(0, tuning_json=text) as ctx:
        for cls, items in graphs.items():
            for name, row, col, w in items:
                g = ctx.graph_load_csr(row, col, w)
                src = autotune.pick_sources(row, 8, seed=5)
                d = ctx.bfs_batch(g, src).cpu().numpy().reshape(src.size, -1)
                s = ctx.sssp_batch(g, src).cpu().numpy().view(np.uint32).reshape(src.size, -1)
                for i in (0, src.size - 1):
                    assert np.array_equal(d[i], oracle.bfs(row, col, src[i])), (name, i)
                    assert np.array_equal(s[i], oracle.sssp(row, col, w, src[i])), (name, i)
                assert np.array_equal(ctx.bfs(g, int(src[1])).cpu().numpy(), oracle.bfs(row, col, src[1]))
                g.free()


def test_class_values_reach_only_their_class():
    import paper_1501_05387_amd as gfr
    graphs = _graphs()
    tuning = {"profile.kernels": 1,
              "scalefree": {"batch.min_bfs": 1},          # shared traversal for any batch
              "mesh": {"batch.min_bfs": 1000}}            # sequential solves
    with gfr.Context(0, tuning_json=json.dumps(tuning)) as ctx:
        loaded = {}
        for cls, items in graphs.items():
            name, row, col, w = items[0]
            loaded[cls] = (ctx.graph_load_csr(row, col, w), row, col)

        def batched(cls):
            g, row, col = loaded[cls]
            src = np.array([0, 1, 2], np.int32)
            d = ctx.bfs_batch(g, src).cpu().numpy().reshape(3, -1)
            assert np.array_equal(d[2], oracle.bfs(row, col, 2))
            try:
                return ctx.stat("t.msbfs_level.n") > 0
            except gfr.GfrError:
                return False

        _say("per-class tuning")
        assert batched("scalefree")
        assert not batched("mesh")
        assert ctx.get_option("batch.min_bfs") == 8          # the context-wide value is untouched
        ctx.set_option("batch.min_bfs", 1)                   # an explicit option beats the file
        assert batched("mesh")
        ctx.set_option("batch.min_bfs", 1000)
        assert not batched("scalefree")
        for g, _, _ in loaded.values():
            g.free()
