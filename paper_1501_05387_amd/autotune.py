"""Autotuner for the frontier engine: sweeps the tuning options on graphs of
each class and writes a tuning file for gfr_ctx_create.

The options it sweeps change only how a result is reached:

* ``advance.chunk``: edges per work-group chunk of the load-balanced advance
  (the partitioned mapping of Sec. 4.4);
* ``bfs.alpha`` / ``bfs.beta``: the push->pull and pull->push switch points of
  direction-optimizing BFS (Sec. 4.5);
* ``sssp.delta_factor``: bucket width of the near/far priority queue
  (Sec. 4.5), as a multiple of the mean edge weight so that it carries over
  between graphs of one class;
* ``msbfs.alpha`` and ``batch.delta_factor``: the same two choices for the
  batched (64 sources at once) traversals, ``batch.blocks_per_cu``, the
  work-groups per CU of the batched relaxation's grid, and ``batch.sparse``,
  the most queries per edge with which a group of edges is relaxed one lane
  per edge rather than one distance row per edge;
* ``batch.min_bfs`` / ``batch.min_sssp``: the batch size from which one
  shared traversal beats sequential single-source solves.

Sec. 7 of the paper fixes such constants by hand and suggests predicting them
from the degree distribution; here the library sorts each graph into a class
("scalefree" or "mesh", by its largest degree against its mean degree) and
the tuner picks the values per class by measurement.

Every candidate's output is compared with the output of the starting
configuration, bit for bit (BFS depths and SSSP distances are unique), so a
setting that changed a result would stop the sweep with an error rather than
be written out.

Usage: ``python -m paper_1501_05387_amd.autotune --out tuning.json`` builds
synthetic R-MAT and grid graphs (the paper's two graph families) and tunes on
them; :func:`tune` takes the caller's own graphs.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import Context

CLASSES = ("scalefree", "mesh")

# candidate values per option (the full sweep and the quick one)
SWEEP = {
    "advance.chunk": [256, 512, 1024, 2048, 4096],
    "bfs.alpha": [2, 5, 10, 15, 30, 60, 120],
    "bfs.beta": [3, 6, 12, 18, 36, 72],
    "sssp.delta_factor": [0.5, 1, 2, 4, 8, 16, 64],
    "msbfs.alpha": [1, 2, 4, 8, 16, 64],
    "batch.delta_factor": [0, 2, 8, 32],
    "batch.blocks_per_cu": [8, 16, 32, 64],
    "batch.sparse": [0, 4, 8, 12],
}
QUICK = {
    "advance.chunk": [512, 2048],
    "bfs.alpha": [5, 30],
    "bfs.beta": [6, 36],
    "sssp.delta_factor": [1, 8],
    "msbfs.alpha": [2, 16],
    "batch.delta_factor": [0, 8],
    "batch.blocks_per_cu": [16, 64],
    "batch.sparse": [0, 8],
}
CROSSOVER_K = [2, 4, 8, 16, 32, 48]
SINGLE_SOURCES = 4          # sources timed per graph for the single-source solvers

DEFAULTS = {
    "advance.chunk": 1024, "bfs.alpha": 15, "bfs.beta": 18, "sssp.delta_factor": 2,
    "msbfs.alpha": 4, "batch.delta_factor": 0, "batch.min_bfs": 8, "batch.min_sssp": 24,
    "batch.blocks_per_cu": 64, "batch.sparse": 8,
}


class NotNeutral(RuntimeError):
    """A tuning option changed a result."""


class _Case:
    """One graph resident on the device, its query sources and reference outputs."""

    def __init__(self, ctx: Context, name: str, row, col, w, sources):
        self.name = name
        self.g = ctx.graph_load_csr(row, col, w)
        self.n = row.size - 1
        self.src = np.asarray(sources, dtype=np.int32)
        self.ref = {}


def pick_sources(row: np.ndarray, count: int, seed: int = 0) -> np.ndarray:
    """Query sources for tuning: the vertex of largest degree, then random
    vertices with at least one edge (deterministic for a seed)."""
    deg = np.diff(row)
    cand = np.nonzero(deg > 0)[0]
    if cand.size == 0:
        return np.zeros(1, np.int32)
    rng = np.random.default_rng(seed)
    pick = rng.choice(cand, size=min(count, cand.size), replace=False)
    out = [int(np.argmax(deg))] + [int(v) for v in pick if v != np.argmax(deg)]
    return np.asarray(out[:count], np.int32)


class Tuner:
    def __init__(self, ctx: Context, repeats: int = 3, log=None):
        self.ctx = ctx
        self.repeats = repeats
        self.log = log or (lambda *a: None)
        import torch
        self.torch = torch

    # ------------------------------------------------------------ measuring
    def _set(self, opts: dict):
        for k, v in opts.items():
            self.ctx.set_option(k, v)

    def _run(self, case: _Case, what: str, k: int | None = None):
        """One solve; returns the device output."""
        c = self.ctx
        if what in ("bfs", "sssp"):
            src = case.src[:SINGLE_SOURCES]
            buf = self._buf(case, len(src))
            solve = c.bfs if what == "bfs" else c.sssp
            for i, v in enumerate(src):
                solve(case.g, int(v), out=buf[i * case.n:(i + 1) * case.n])
            return buf
        src = case.src[:k]
        if what == "bfs_batch":
            return c.bfs_batch(case.g, src, out=self._buf(case, len(src)))
        return c.sssp_batch(case.g, src, out=self._buf(case, len(src)))

    def _buf(self, case: _Case, rows: int):
        key = ("buf", rows)
        if key not in case.ref:
            case.ref[key] = self.torch.empty(rows * case.n, dtype=self.torch.int32, device="cuda:%d" % self.ctx.device)
        return case.ref[key]

    def _time(self, case: _Case, what: str, k: int | None = None) -> float:
        """Median wall time of a solve (seconds), after checking its output."""
        torch = self.torch
        out = self._run(case, what, k)                       # warm-up and neutrality check
        torch.cuda.synchronize()
        ref_key = (what, k)
        if ref_key not in case.ref:
            case.ref[ref_key] = out.clone()
        elif not torch.equal(out, case.ref[ref_key]):
            raise NotNeutral("%s on %s (k=%s) changed its result" % (what, case.name, k))
        ts = []
        for _ in range(self.repeats):
            t0 = time.perf_counter()
            self._run(case, what, k)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def _cost(self, cases, whats, opts, k=None) -> float:
        self._set(opts)
        return sum(self._time(c, w, k) for c in cases for w in whats)

    def _descend(self, cases, whats, keys, sweep, opts, k=None, rounds=2) -> dict:
        """Coordinate descent over `keys`, starting from `opts`, on the summed
        time of the solves in `whats`."""
        best = dict(opts)
        best_t = self._cost(cases, whats, best, k)
        for _ in range(rounds):
            moved = False
            for key in keys:
                for v in sweep[key]:
                    if v == best[key]:
                        continue
                    trial = dict(best, **{key: v})
                    t = self._cost(cases, whats, trial, k)
                    if t < best_t * 0.98:                       # 2 % to beat noise
                        best, best_t, moved = trial, t, True
                self.log("  %s %s -> %s (%.3f ms)" % ("+".join(whats), key, best[key], best_t * 1e3))
            if not moved:
                break
        self._set(best)
        return best

    def _crossover(self, cases, what) -> int:
        """Smallest batch size from which one shared traversal beats
        sequential single-source solves."""
        key = "batch.min_bfs" if what == "bfs_batch" else "batch.min_sssp"
        for k in CROSSOVER_K:
            if any(c.src.size < k for c in cases):
                break
            self.ctx.set_option(key, 1)
            shared = sum(self._time(c, what, k) for c in cases)
            self.ctx.set_option(key, 10 ** 9)
            seq = sum(self._time(c, what, k) for c in cases)
            self.log("  %s k=%d shared %.3f ms sequential %.3f ms" % (what, k, shared * 1e3, seq * 1e3))
            if shared < seq:
                self.ctx.set_option(key, k)
                return k
        self.ctx.set_option(key, 65)         # sequential solves won at every size tried
        return 65

    # --------------------------------------------------------------- driver
    def tune_class(self, cases, quick: bool = False) -> dict:
        sweep = QUICK if quick else SWEEP
        opts = dict(DEFAULTS)
        self._set(opts)
        weighted = all(c.g.weighted for c in cases)
        opts = self._descend(cases, ["bfs"], ["bfs.alpha", "bfs.beta"], sweep, opts)
        if weighted:
            opts = self._descend(cases, ["sssp"], ["sssp.delta_factor"], sweep, opts)
        # the chunk serves every advance: tune it on the sum
        opts = self._descend(cases, ["bfs", "sssp"] if weighted else ["bfs"], ["advance.chunk"], sweep, opts,
                             rounds=1)
        kmax = min(64, min(c.src.size for c in cases))
        opts = self._descend(cases, ["bfs_batch"], ["msbfs.alpha"], sweep, dict(opts, **{"batch.min_bfs": 1}),
                             k=kmax, rounds=1)
        if weighted:
            opts = self._descend(cases, ["sssp_batch"], ["batch.delta_factor", "batch.blocks_per_cu", "batch.sparse"], sweep,
                                 dict(opts, **{"batch.min_sssp": 1}), k=kmax, rounds=1)
        opts["batch.min_bfs"] = self._crossover(cases, "bfs_batch")
        if weighted:
            opts["batch.min_sssp"] = self._crossover(cases, "sssp_batch")
        return opts


def tune(ctx: Context, graphs: dict, quick: bool = False, repeats: int = 3, sources: int = 64, log=None) -> dict:
    """Tune per graph class.

    graphs: {class name: [(name, row, col, weights or None), ...]} with class
    names from CLASSES.  Options set on `ctx` are overwritten during the sweep
    and restored at the end.  Returns the tuning file's content as a dict
    ({class: {option: value}}).
    """
    keys = list(DEFAULTS)
    saved = {k: ctx.get_option(k) for k in keys}
    tuner = Tuner(ctx, repeats=repeats, log=log)
    result = {}
    try:
        for cls, items in graphs.items():
            if cls not in CLASSES:
                raise ValueError("unknown graph class %r (expected one of %s)" % (cls, CLASSES))
            cases = [_Case(ctx, name, row, col, w, pick_sources(row, sources, seed=i))
                     for i, (name, row, col, w) in enumerate(items)]
            try:
                (log or (lambda *a: None))("class %s: %s" % (cls, ", ".join(c.name for c in cases)))
                result[cls] = tuner.tune_class(cases, quick=quick)
            finally:
                for c in cases:
                    c.g.free()
    finally:
        for k, v in saved.items():
            ctx.set_option(k, v)
    return result


def _synthetic(scales, grid_side):
    import graphgen
    out = {"scalefree": [], "mesh": []}
    for s in scales:
        row, col = graphgen.rmat(s, 16)
        out["scalefree"].append(("rmat%d" % s, row, col, graphgen.weights(row, col, 64)))
    row, col = graphgen.grid(grid_side)
    out["mesh"].append(("grid%d" % grid_side, row, col, graphgen.weights(row, col, 1000)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default="tuning.json")
    ap.add_argument("--scales", default="16,20,22", help="R-MAT scales of the scale-free class")
    ap.add_argument("--grid", type=int, default=4096, help="side of the grid graph of the mesh class")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--repeats", type=int, default=3)
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    graphs = _synthetic([int(s) for s in a.scales.split(",") if s], a.grid)
    ctx = Context(0)
    res = tune(ctx, graphs, quick=a.quick, repeats=a.repeats, log=log)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(res, sort_keys=True))


if __name__ == "__main__":
    main()
