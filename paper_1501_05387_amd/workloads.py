"""One traversal mode at a time, for profiler runs.

``python -m paper_1501_05387_amd.workloads --mode MODE [--scale 22] [--reps 3]``
loads the seeded R-MAT graph of the benchmark (edge factor 16, weights in
[1,64]) or the 4096^2 lattice (``--graph grid``), warms up once, then runs the
mode ``reps`` times and prints one line per run with its device time.  Under
``rocprofv3 --kernel-trace --stats`` or ``--pmc`` this isolates the kernels of
one mode:

    push_bfs      single-source BFS forced to push (bfs_level + compaction)
    do_bfs        single-source direction-optimizing BFS
    sssp          single-source SSSP (sssp_relax + compaction)
    msbfs         64-source batched BFS (msbfs_level, msbfs_finalize, ...)
    bsssp         64-query batched SSSP (bsssp_relax + bsssp_compact)
    copy          a 1 GiB elementwise kernel (bitwise_not: reads and writes
                  1 GiB) and a 1 GiB sum (reads 1 GiB): known sizes that
                  calibrate the byte counters

Sources are the first of the 64 the benchmark draws (seed 3).
"""
from __future__ import annotations

import argparse
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--mode", required=True,
                    choices=["push_bfs", "do_bfs", "sssp", "msbfs", "bsssp", "copy"])
    ap.add_argument("--graph", default="rmat", choices=["rmat", "grid"])
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)

    import torch

    import graphgen
    import paper_1501_05387_amd as gfr

    def say(*a):
        print("[workload]", *a, flush=True)

    if args.mode == "copy":
        nw = (1 << 30) // 4
        a = torch.ones(nw, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(args.reps):
            torch.bitwise_not(a, out=b)
            tot = int(torch.sum(a).item())
        torch.cuda.synchronize()
        say("copy: %d x (bitwise_not over 1 GiB, sum over 1 GiB = %d)" % (args.reps, tot))
        return 0

    if args.graph == "rmat":
        row, col = graphgen.rmat(args.scale, 16)
        w = graphgen.weights(row, col, 64)
    else:
        row, col = graphgen.grid(4096)
        w = graphgen.weights(row, col, 1000)
    srcs = graphgen.sample_sources(row, col, 64)
    n = row.size - 1
    ctx = gfr.Context(0, tuning_json=gfr.tuned_json())
    g = ctx.graph_load_csr(row, col, w)
    say("%s n=%d m=%d mode %s" % (args.graph, n, col.size, args.mode))
    if args.mode == "push_bfs":
        ctx.set_option("bfs.direction", 1)
        ctx.set_option("bfs.frontier", 1)
    out = torch.empty(64 * n, dtype=torch.int32, device="cuda:0")

    def run(i):
        s = int(srcs[i % 64])
        if args.mode in ("push_bfs", "do_bfs"):
            ctx.bfs(g, s, out=out[:n])
        elif args.mode == "sssp":
            ctx.sssp(g, s, out=out[:n])
        elif args.mode == "msbfs":
            ctx.bfs_batch(g, srcs, out=out)
        else:
            ctx.sssp_batch(g, srcs, out=out)

    run(0)
    torch.cuda.synchronize()
    for i in range(args.reps):
        t = time.perf_counter()
        run(i + 1)
        say("run %d: %.3f ms (device %.3f ms)" % (i, (time.perf_counter() - t) * 1e3, ctx.stat("kernel_ms")))
    g.free()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
