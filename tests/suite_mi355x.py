"""The measurement suite: every measurement row on one MI355X, with parity
samples and error reports against the CPU oracle.

    python -m tests.suite_mi355x --out profiles/suite_mi355x.json    (about 4 minutes)

Rows: R-MAT s16 BFS launch overhead; the R-MAT s22 modes (push BFS,
direction-optimizing BFS, SSSP, 64-source MS-BFS and batched SSSP) with GTEPS
distributions and algorithmic GB/s; the 4096^2 lattice (push/pull log, SSSP
re-relaxation, CC); R-MAT s23 PageRank, filtered PageRank and BC; the
filtered-PageRank error report on R-MAT s20; 2-hop, personalized PageRank,
SALSA and HITS; the six-graph serving ladder.  It sits with the tests because
its checks call the oracle; the timed work is the engine's alone, and the byte
models and the serving leg are the benchmark's own (bench.py).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from bench import (HBM_PEAK_GBS, STAT_KEYS, SERVE_SCALES, bfs_bytes, bsssp_floor_bytes,  # noqa: E402
                   kernel_source_digest, msbfs_bytes, read_stats, serve_leg, sssp_bytes)


def _dist(vals):
    v = np.asarray(vals, dtype=np.float64)
    return {"hmean": float(len(v) / np.sum(1.0 / v)), "p25": float(np.percentile(v, 25)),
            "p50": float(np.percentile(v, 50)), "p75": float(np.percentile(v, 75)),
            "min": float(v.min()), "max": float(v.max())}


def _timed(ctx, fn, reps, warm=2):
    """Device times (kernel_ms of each call) of `reps` calls after `warm` calls."""
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        fn()
        ts.append(ctx.stat("kernel_ms"))
    return ts


PRF_TOLS = (1e-2, 1e-4, 1e-6)   # filtered PageRank tolerances, in units of 1/N


def prf_error_report(ctx, log, scale=20):
    """Filtered PageRank on R-MAT s20 against the FP64 fixed point (the oracle
    run until its L1 change is below 1e-11): L1 error, iterations and the share
    of vertex updates per tolerance, beside plain FP32 power iteration to 1e-6."""
    import graphgen
    import oracle
    row, col = graphgen.rmat(scale)
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    xs, its, _ = oracle.pagerank(row, col, 0.85, 1e-11, 10000)
    rep = {"fixed_point_iterations": its}
    x, it, _ = ctx.pagerank(g, 0.85, 1e-6, 1000)
    rep["plain_fp32_tol1e-6"] = {"iterations": it, "l1_error": float(np.abs(x.cpu().numpy() - xs).sum())}
    for c in PRF_TOLS:
        x, _, it, _ = ctx.pagerank_filtered(g, 0.85, c / n, 1000)
        rep["%g/N" % c] = {"iterations": it, "l1_error": float(np.abs(x.cpu().numpy() - xs).sum()),
                           "vertex_update_share": ctx.stat("vertex_updates") / (it * n)}
    log("d4 filtered pagerank error report", rep)
    g.free()
    return rep


def rank_leg(ctx, log):
    """2-hop walk counts on R-MAT s22 (1 and 64 seeds, both directions of the
    second advance), personalized PageRank on R-MAT s22 from 1 and 64 seeds,
    SALSA and HITS on a bipartite R-MAT with 2^21 vertices per side; each with
    a parity sample against the oracle."""
    import graphgen
    import oracle
    out = {}
    row, col = graphgen.rmat(22)
    n = row.size - 1
    g = ctx.graph_load_csr(row, col)
    seeds64 = graphgen.sample_sources(row, col, 64)
    for k in (1, 64):
        S = seeds64[:k]
        for direction, name in ((1, "push"), (2, "pull"), (0, "auto")):
            ctx.set_option("twohop.direction", direction)
            ts = _timed(ctx, lambda: ctx.two_hop(g, S), 5)
            e = ctx.stat("edges_inspected")
            out["two_hop_%d_%s" % (k, name)] = {"ms_median": float(np.median(ts)), "edges_inspected": e,
                                               "gteps": e / (float(np.median(ts)) * 1e-3) / 1e9}
            log("d6 two_hop", k, name, out["two_hop_%d_%s" % (k, name)])
        ctx.set_option("twohop.direction", 0)
        got = ctx.two_hop(g, S).cpu().numpy().view(np.uint64)
        out["two_hop_%d_bit_exact" % k] = bool(np.array_equal(got, oracle.two_hop(row, col, S)))
    for k in (1, 64):
        S = seeds64[:k]
        ts = _timed(ctx, lambda: ctx.ppr(g, S, 0.85, 1e-9, 1000), 3, warm=1)
        x, it, l1 = ctx.ppr(g, S, 0.85, 1e-9, 1000)
        out["ppr_%d" % k] = {"ms_median": float(np.median(ts)), "iterations": it,
                             "ms_per_iteration": float(np.median(ts)) / it}
        log("d6 ppr", k, out["ppr_%d" % k])
    xo, _, _ = oracle.ppr(row, col, seeds64[:1], 0.85, 0.0, out["ppr_1"]["iterations"])
    x, _, _ = ctx.ppr(g, seeds64[:1], 0.85, 1e-9, 1000)
    out["ppr_1_l1_vs_oracle"] = float(np.abs(x.cpu().numpy() - xo).sum())
    g.free()
    del row, col
    row, col = graphgen.bipartite_rmat(21)
    nl = 1 << 21
    g = ctx.graph_load_csr(row, col)
    for method in ("salsa", "hits"):
        fn = getattr(ctx, method)
        ts = _timed(ctx, lambda: fn(g, nl, 20), 3, warm=1)
        out[method + "_20_iterations"] = {"ms_median": float(np.median(ts)),
                                          "ms_per_iteration": float(np.median(ts)) / 20,
                                          "edges_per_s": 20 * col.size / (float(np.median(ts)) * 1e-3)}
        h, a = fn(g, nl, 5)
        ho, ao = getattr(oracle, method)(row, col, nl, 5)
        out[method + "_5_max_abs_err"] = float(max(np.abs(h.cpu().numpy() - ho).max(), np.abs(a.cpu().numpy() - ao).max()))
        log("d6", method, out[method + "_20_iterations"], out[method + "_5_max_abs_err"])
    out["bipartite_graph"] = {"n": int(row.size - 1), "m": int(col.size)}
    g.free()
    return out


def suite(args, log):
    """The measurement rows of the design: R-MAT s16 BFS launch overhead; the
    R-MAT s22 modes (push BFS, direction-optimizing BFS, SSSP, 64-source
    MS-BFS and batched SSSP) with GTEPS distributions and algorithmic GB/s;
    the 4096^2 lattice (thin frontiers, push/pull log, SSSP re-relaxation,
    CC); R-MAT s23 PageRank and BC with their errors against the oracle; the
    six-graph serving ladder.  Times are device times of whole calls
    (median and mean of 10 after 2 warm-ups unless stated)."""
    import torch

    import graphgen
    import oracle
    import paper_1501_05387_amd as gfr
    ctx = gfr.Context(0, tuning_json=gfr.tuned_json())
    rep = {"device": torch.cuda.get_device_name(0), "host_cpus": os.cpu_count(),
           "source_digest": kernel_source_digest(), "peak_hbm_GBs": HBM_PEAK_GBS}

    def te_of(row, depth):
        return int(np.diff(row)[depth >= 0].sum())

    if "1" in args.suite_parts:
        # d.1 R-MAT s16 BFS from vertex 0
        row, col = graphgen.rmat(16)
        g = ctx.graph_load_csr(row, col)
        ok = bool(np.array_equal(ctx.bfs(g, 0).cpu().numpy(), oracle.bfs(row, col, 0)))
        ts = _timed(ctx, lambda: ctx.bfs(g, 0), 10)
        lv = ctx.stat("levels")
        rep["d1_rmat16_bfs0"] = {"bit_exact": ok, "ms_median": float(np.median(ts)), "ms_mean": float(np.mean(ts)),
                                 "levels": lv, "us_per_level": float(np.median(ts)) * 1e3 / max(lv, 1),
                                 "gteps": te_of(row, oracle.bfs(row, col, 0)) / (np.median(ts) * 1e-3) / 1e9}
        log("d1", rep["d1_rmat16_bfs0"])
        g.free()

    if "2" in args.suite_parts:
        # d.2 R-MAT s22, 64 sources
        row, col = graphgen.rmat(22)
        w = graphgen.weights(row, col, 64)
        n = row.size - 1
        srcs = graphgen.sample_sources(row, col, 64)
        g = ctx.graph_load_csr(row, col, w)
        dep = ctx.bfs_batch(g, srcs).view(64, n).cpu().numpy()
        te = np.array([te_of(row, dep[i]) for i in range(64)], dtype=np.float64)
        d2 = {}
        for mode, direction, frontier in (("push_bfs", 1, 0), ("do_bfs", 0, 0), ("queue_push_bfs", 1, 1),
                                          ("queue_do_bfs", 0, 1)):
            ctx.set_option("bfs.direction", direction)
            ctx.set_option("bfs.frontier", frontier)
            gt, gbs, lvls = [], [], []
            for i, sidx in enumerate(srcs):
                ts = _timed(ctx, lambda: ctx.bfs(g, int(sidx)), 10, warm=1)
                st = read_stats(ctx, STAT_KEYS)
                t = float(np.median(ts)) * 1e-3
                gt.append(te[i] / t / 1e9)
                gbs.append(bfs_bytes(st, 1, n) / t / 1e9)
                lvls.append(st.get("levels", 0))
            d2[mode] = {"gteps": _dist(gt), "gteps_graph500": _dist(np.array(gt) / 2), "alg_GBs": _dist(gbs),
                        "alg_frac_of_peak_p50": float(np.median(gbs)) / HBM_PEAK_GBS, "levels_p50": float(np.median(lvls))}
            log("d2", mode, d2[mode]["gteps"])
        ctx.set_option("bfs.direction", 0)
        ctx.set_option("bfs.frontier", 0)
        gt, gbs, rr = [], [], []
        for i, sidx in enumerate(srcs):
            ts = _timed(ctx, lambda: ctx.sssp(g, int(sidx)), 10, warm=1)
            st = read_stats(ctx, STAT_KEYS)
            t = float(np.median(ts)) * 1e-3
            gt.append(te[i] / t / 1e9)
            gbs.append(sssp_bytes(st) / t / 1e9)
            rr.append(st["relaxations"] / te[i])
        d2["sssp"] = {"gteps": _dist(gt), "gteps_graph500": _dist(np.array(gt) / 2), "alg_GBs": _dist(gbs),
                      "alg_frac_of_peak_p50": float(np.median(gbs)) / HBM_PEAK_GBS, "rerelaxation_r": _dist(rr)}
        log("d2 sssp", d2["sssp"]["gteps"])
        for mode, fn, bytes_of in (("msbfs_64", lambda: ctx.bfs_batch(g, srcs), lambda st: msbfs_bytes(dict(st, m=g.m), n)),
                                   ("batched_sssp_64", lambda: ctx.sssp_batch(g, srcs),
                                    lambda st: bsssp_floor_bytes(int((dep >= 0).sum()), int(te.sum()), 64))):
            ts = _timed(ctx, fn, 10)
            st = read_stats(ctx, STAT_KEYS)
            t = float(np.median(ts)) * 1e-3
            d2[mode] = {"ms_median": t * 1e3, "ms_mean": float(np.mean(ts)), "gteps": float(te.sum() / t / 1e9),
                        "gteps_graph500": float(te.sum() / 2 / t / 1e9), "alg_GBs": bytes_of(st) / t / 1e9,
                        "alg_frac_of_peak": bytes_of(st) / t / 1e9 / HBM_PEAK_GBS}
            log("d2", mode, d2[mode])
        par = all(np.array_equal(ctx.sssp(g, int(srcs[i])).cpu().numpy().view(np.uint32), oracle.sssp(row, col, w, srcs[i]))
                  for i in (0, 63))
        d2["parity_sample_ok"] = bool(par and all(np.array_equal(dep[i], oracle.bfs(row, col, srcs[i])) for i in (0, 63)))
        rep["d2_rmat22"] = d2
        g.free()
        del row, col, w, dep

    if "3" in args.suite_parts:
        # d.3 4096^2 lattice, 16 sources
        row, col = graphgen.grid(4096)
        w = graphgen.weights(row, col, 1000)
        srcs = graphgen.sample_sources(row, col, 16)
        g = ctx.graph_load_csr(row, col, w)
        d3 = {}
        for mode, direction, frontier in (("push_bfs", 1, 0), ("do_bfs", 0, 0), ("queue_push_bfs", 1, 1),
                                          ("queue_do_bfs", 0, 1)):
            ctx.set_option("bfs.direction", direction)
            ctx.set_option("bfs.frontier", frontier)
            gt, upl, logs = [], [], []
            for sidx in srcs:
                ts = _timed(ctx, lambda: ctx.bfs(g, int(sidx)), 3, warm=1)
                st = read_stats(ctx, STAT_KEYS)
                t = float(np.median(ts))
                d = ctx.bfs(g, int(sidx)).cpu().numpy()
                gt.append(te_of(row, d) / (t * 1e-3) / 1e9)
                upl.append(t * 1e3 / max(st.get("levels", 1), 1))
                logs.append((int(st.get("levels", 0)), int(ctx.stat("push_levels")), int(st.get("pull_levels", 0))))
            d3[mode] = {"gteps": _dist(gt), "us_per_level": _dist(upl), "levels_push_pull": logs[:4]}
            log("d3", mode, d3[mode]["gteps"], d3[mode]["us_per_level"])
        ctx.set_option("bfs.direction", 0)
        gt, rr = [], []
        for sidx in srcs:
            ts = _timed(ctx, lambda: ctx.sssp(g, int(sidx)), 3, warm=1)
            st = read_stats(ctx, STAT_KEYS)
            d = ctx.bfs(g, int(sidx)).cpu().numpy()
            tsum = te_of(row, d)
            gt.append(tsum / (float(np.median(ts)) * 1e-3) / 1e9)
            rr.append(st["relaxations"] / tsum)
        d3["sssp"] = {"gteps": _dist(gt), "rerelaxation_r": _dist(rr)}
        ts = _timed(ctx, lambda: ctx.cc(g), 10)
        lab, k = ctx.cc(g)
        ref, kref = oracle.cc(row, col)
        d3["cc"] = {"ms_median": float(np.median(ts)), "components": k, "bit_exact": bool(np.array_equal(lab.cpu().numpy(), ref))}
        d3["parity_sample_ok"] = bool(np.array_equal(ctx.bfs(g, int(srcs[0])).cpu().numpy(), oracle.bfs(row, col, srcs[0])) and
                                      np.array_equal(ctx.sssp(g, int(srcs[0])).cpu().numpy().view(np.uint32),
                                                     oracle.sssp(row, col, w, srcs[0])))
        log("d3 sssp/cc", d3["sssp"]["gteps"], d3["cc"])
        rep["d3_grid4096"] = d3
        g.free()
        del row, col, w

    if "4" in args.suite_parts:
        # d.4 R-MAT s23 PageRank and BC
        row, col = graphgen.rmat(23)
        n = row.size - 1
        g = ctx.graph_load_csr(row, col)
        ts = _timed(ctx, lambda: ctx.pagerank(g, 0.85, 1e-6, 1000), 3, warm=1)
        x, it, l1 = ctx.pagerank(g, 0.85, 1e-6, 1000)
        xo, _, _ = oracle.pagerank(row, col, 0.85, 0.0, it)
        pr_err = float(np.abs(x.cpu().numpy().astype(np.float64) - xo).sum())
        d4 = {"pagerank": {"ms_median": float(np.median(ts)), "iterations": it, "ms_per_iteration": float(np.median(ts)) / it,
                           "final_l1": l1, "l1_vs_fp64_oracle": pr_err}}
        log("d4 pagerank", d4["pagerank"])
        # per-vertex convergence filtering: time and work per tolerance (units of 1/N)
        d4["pagerank_filtered"] = {}
        for c in PRF_TOLS:
            ts = _timed(ctx, lambda: ctx.pagerank_filtered(g, 0.85, c / n, 1000), 3, warm=1)
            st = read_stats(ctx, ("iterations", "vertex_updates", "edges_gathered"))
            itf = st["iterations"]
            d4["pagerank_filtered"]["%g/N" % c] = {
                "ms_median": float(np.median(ts)), "iterations": itf,
                "vertex_update_share": st["vertex_updates"] / (itf * n),
                "edge_share": st["edges_gathered"] / (itf * g.m)}
            log("d4 pagerank_filtered", c, d4["pagerank_filtered"]["%g/N" % c])
        src32 = graphgen.sample_sources(row, col, 32)
        ts = _timed(ctx, lambda: ctx.bc(g, src32), 2, warm=1)
        d32 = ctx.bfs_batch(g, src32).view(32, n).cpu().numpy()
        te32 = sum(te_of(row, d32[i]) for i in range(32))
        bc32 = ctx.bc(g, src32).cpu().numpy().astype(np.float64)
        ident = float(sum(np.sum(d32[i][d32[i] > 0] - 1, dtype=np.float64) for i in range(32)))
        bc4 = ctx.bc(g, src32[:4]).cpu().numpy().astype(np.float64)
        ref4 = oracle.bc(row, col, src32[:4])
        nz = ref4 != 0
        d4["bc_32"] = {"ms_median": float(np.median(ts)), "gteps_2x": 2.0 * te32 / (float(np.median(ts)) * 1e-3) / 1e9,
                       "max_rel_err_4_sources": float(np.max(np.abs(bc4 - ref4) / np.maximum(np.abs(ref4), 1.0))),
                       "mean_rel_err_4_sources": float(np.mean(np.abs(bc4[nz] - ref4[nz]) / ref4[nz])),
                       "zero_where_oracle_zero": bool(np.all(bc4[~nz] == 0)),
                       "identity_rel_residual_32": abs(float(bc32.sum()) - ident) / ident}
        log("d4 bc", d4["bc_32"])
        rep["d4_rmat23"] = d4
        g.free()
        del row, col
        rep["d4_rmat20_pagerank_filtered_error"] = prf_error_report(ctx, log)

    if "6" in args.suite_parts:
        # d.6 the 2-hop advance and the node rankings
        rep["d6_two_hop_and_ranking"] = rank_leg(ctx, log)

    if "5" in args.suite_parts:
        # d.5 serving ladder
        resident = {}
        for sc in SERVE_SCALES:
            r2, c2 = graphgen.rmat(sc, 16)
            w2 = graphgen.weights(r2, c2, 64)
            resident[sc] = (r2, c2, w2, ctx.graph_load_csr(r2, c2, w2))
        rep["d5_serving"] = serve_leg(ctx, resident, args.suite_queries, log, rates=(500.0, 2000.0, 8000.0, 16000.0, 1e9))
        for sc, (_, _, _, g2) in resident.items():
            g2.free()
    ctx.close()
    return rep


def render_md(rep) -> str:
    """The suite's report as markdown tables (the figures of `rep`, nothing else)."""
    L = ["# Measurement suite on one MI355X", "",
         "Command (repository root): `python -m tests.suite_mi355x --out profiles/suite_mi355x.json --md "
         "profiles/suite_mi355x.md` (about 3 minutes). Device times of whole calls; median of 10 after warm-up unless "
         "stated; GTEPS = sum of degrees of reached vertices / time (Graph500 count = half). Algorithmic GB/s from the "
         "kernels' own counters (byte models in the design notes); for the batched SSSP from the SSSP work model at r = "
         "1, which its 64 results fix; against 8 TB/s.",
         "Kernel sources digest `%s`; device %s." % (rep.get("source_digest"), rep.get("device"))]
    d1 = rep.get("d1_rmat16_bfs0")
    if d1:
        L += ["", "## R-MAT s16, BFS from vertex 0", "", "| bit-exact | ms | levels | µs per level | GTEPS |",
              "|---|---|---|---|---|",
              "| %s | %.3f | %d | %.1f | %.1f |" % (d1["bit_exact"], d1["ms_median"], d1["levels"], d1["us_per_level"],
                                                d1["gteps"])]
    d2 = rep.get("d2_rmat22")
    if d2:
        L += ["", "## R-MAT s22, 64 sources (parity sample ok: %s)" % d2["parity_sample_ok"], "",
              "| mode | GTEPS hmean | p25 / p50 / p75 | alg GB/s (p50) | of peak |", "|---|---|---|---|---|"]
        for mode in ("push_bfs", "do_bfs", "queue_push_bfs", "queue_do_bfs", "sssp"):
            r = d2[mode]
            L.append("| %s (per source) | %.1f | %.1f / %.1f / %.1f | %.0f | %.3f |" % (
                mode, r["gteps"]["hmean"], r["gteps"]["p25"], r["gteps"]["p50"], r["gteps"]["p75"],
                r["alg_GBs"]["p50"], r["alg_frac_of_peak_p50"]))
        for mode in ("msbfs_64", "batched_sssp_64"):
            r = d2[mode]
            L.append("| %s (one call, %.2f ms) | %.1f (aggregate) | — | %.0f | %.3f |" % (
                mode, r["ms_median"], r["gteps"], r["alg_GBs"], r["alg_frac_of_peak"]))
        L += ["", "Single-source SSSP re-relaxation factor r (edges relaxed / edges of reached vertices): p50 %.2f."
              % d2["sssp"]["rerelaxation_r"]["p50"]]
    d3 = rep.get("d3_grid4096")
    if d3:
        L += ["", "## 4096² lattice with long edges, 16 sources (parity sample ok: %s)" % d3["parity_sample_ok"], "",
              "| mode | GTEPS hmean | µs per level (p50) | levels / push / pull (first sources) |", "|---|---|---|---|"]
        names = {"push_bfs": "push_bfs (mark-byte levels, the mesh default)", "do_bfs": "do_bfs (auto: mark-byte levels)",
                 "queue_push_bfs": "push_bfs, queue levels", "queue_do_bfs": "do_bfs, queue levels"}
        for mode, label in names.items():
            r = d3[mode]
            L.append("| %s | %.2f | %.1f | %s |" % (label, r["gteps"]["hmean"], r["us_per_level"]["p50"],
                                                  r["levels_push_pull"]))
        L.append("| sssp | %.2f | — | r p50 %.2f |" % (d3["sssp"]["gteps"]["hmean"], d3["sssp"]["rerelaxation_r"]["p50"]))
        L += ["", "CC: %.2f ms, %d components, bit-exact %s." % (d3["cc"]["ms_median"], d3["cc"]["components"],
                                                                 d3["cc"]["bit_exact"])]
    d4 = rep.get("d4_rmat23")
    if d4:
        pr = d4["pagerank"]
        L += ["", "## R-MAT s23", "",
              "PageRank (d = 0.85, L1 < 1e-6): %.1f ms, %d iterations, %.2f ms per iteration, final L1 %.2e, L1 against "
              "the FP64 oracle at the same iteration count %.2e." % (pr["ms_median"], pr["iterations"],
                                                                     pr["ms_per_iteration"], pr["final_l1"],
                                                                     pr["l1_vs_fp64_oracle"]), "",
              "PageRank with per-vertex convergence filtering (FP64), per tolerance in units of 1/N:", "",
              "| vertex_tol | ms | iterations | vertex updates / (iterations × N) | edges gathered / (iterations × m) |",
              "|---|---|---|---|---|"]
        for k, r in d4["pagerank_filtered"].items():
            L.append("| %s | %.1f | %d | %.3f | %.3f |" % (k, r["ms_median"], r["iterations"], r["vertex_update_share"],
                                                          r["edge_share"]))
        b = d4["bc_32"]
        L += ["", "BC from 32 sources: %.1f ms, %.1f GTEPS (2× convention); against the oracle on 4 sources largest "
              "relative error %.2e, mean %.2e, zero wherever the oracle is zero: %s; path-length identity over all 32 "
              "sources (sum of BC = sum of d(s,t) - 1) holds to a relative residual of %.1e." % (
                  b["ms_median"], b["gteps_2x"], b["max_rel_err_4_sources"], b["mean_rel_err_4_sources"],
                  b["zero_where_oracle_zero"], b["identity_rel_residual_32"])]
    pe = rep.get("d4_rmat20_pagerank_filtered_error")
    if pe:
        L += ["", "## Filtered PageRank error report, R-MAT s20", "",
              "Against the FP64 fixed point (oracle until its L1 change is below 1e-11, %d iterations):"
              % pe["fixed_point_iterations"], "",
              "| run | iterations | L1 error | vertex updates / (iterations × N) |", "|---|---|---|---|",
              "| plain FP32, L1 < 1e-6 | %d | %.2e | 1 |" % (pe["plain_fp32_tol1e-6"]["iterations"],
                                                          pe["plain_fp32_tol1e-6"]["l1_error"])]
        for k, r in pe.items():
            if k.endswith("/N"):
                L.append("| filtered, vertex_tol %s | %d | %.2e | %.3f |" % (k, r["iterations"], r["l1_error"],
                                                                           r["vertex_update_share"]))
    d6 = rep.get("d6_two_hop_and_ranking")
    if d6:
        L += ["", "## 2-hop walk counts and node rankings", "",
              "R-MAT s22. 2-hop from 1 and 64 seeds, each direction of the second advance (bit-exact against the "
              "oracle: %s, %s):" % (d6["two_hop_1_bit_exact"], d6["two_hop_64_bit_exact"]), "",
              "| seeds | direction | ms | edges inspected | G edges/s |", "|---|---|---|---|---|"]
        for seeds in (1, 64):
            for dr in ("push", "pull", "auto"):
                r = d6["two_hop_%d_%s" % (seeds, dr)]
                L.append("| %d | %s | %.3f | %.3g | %.1f |" % (seeds, dr, r["ms_median"], r["edges_inspected"], r["gteps"]))
        L += ["", "Personalized PageRank (FP64, L1 < 1e-9): 1 seed %.1f ms (%d iterations, %.2f ms each), 64 seeds "
              "%.1f ms; L1 against the oracle %.1e." % (d6["ppr_1"]["ms_median"], d6["ppr_1"]["iterations"],
                                                        d6["ppr_1"]["ms_per_iteration"], d6["ppr_64"]["ms_median"],
                                                        d6["ppr_1_l1_vs_oracle"]), "",
              "Bipartite R-MAT, 2^21 vertices per side (n = %d, m = %d directed entries), 20 iterations:"
              % (d6["bipartite_graph"]["n"], d6["bipartite_graph"]["m"]), "",
              "| method | ms | ms per iteration | G edges/s | max abs error vs oracle (5 iterations) |",
              "|---|---|---|---|---|"]
        for name, key in (("SALSA", "salsa"), ("HITS", "hits")):
            r = d6["%s_20_iterations" % key]
            L.append("| %s | %.2f | %.3f | %.1f | %.1e |" % (name, r["ms_median"], r["ms_per_iteration"],
                                                           r["edges_per_s"] / 1e9, d6["%s_5_max_abs_err" % key]))
    d5 = rep.get("d5_serving")
    if d5:
        L += ["", "## Serving: six R-MAT graphs s18-s23, %d queries per point" % d5["queries_per_point"], "",
              d5["mix"] + ".", "",
              "| offered q/s | batched q/s | p50 / p99 ms | lanes per step | joined running | equal | one at a time q/s "
              "| p50 / p99 ms |", "|---|---|---|---|---|---|---|---|"]
        for b, o in zip(d5["batched"], d5["one_at_a_time"]):
            L.append("| %s | %.0f | %.1f / %.1f | %.1f | %d | %s | %.0f | %.1f / %.1f |" % (
                "burst" if b["offered_qps"] is None else "%.0f" % b["offered_qps"], b["qps"], b["p50_ms"], b["p99_ms"],
                b["mean_batch"], b["joined_running"], b["results_equal"] and o["results_equal"], o["qps"], o["p50_ms"],
                o["p99_ms"]))
    return "\n".join(L) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="write the suite's JSON here")
    ap.add_argument("--suite-queries", type=int, default=10000, help="serving queries per point")
    ap.add_argument("--suite-parts", default="123456", help="rows to run (digits of d.1 .. d.6)")
    ap.add_argument("--md", help="also write the report as markdown here")
    ap.add_argument("--render", action="store_true", help="only render the JSON at --out as markdown (--md)")
    args = ap.parse_args()
    if args.render:
        with open(args.md, "w") as f:
            f.write(render_md(json.load(open(args.out))))
        return

    def log(*a):
        print("[suite]", *a, file=sys.stderr, flush=True)

    rep = suite(args, log)
    with open(args.out, "w") as f:
        json.dump(rep, f, indent=1)
    if args.md:
        with open(args.md, "w") as f:
            f.write(render_md(rep))
    log("suite written to", args.out)


if __name__ == "__main__":
    main()
