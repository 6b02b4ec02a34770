"""Independent oracle solves run side by side, one single-threaded oracle call
per worker thread.

The oracle's C functions hold no global state and ctypes releases the GIL
for the duration of a foreign call, so each thread runs one plain
single-threaded solve at a time; results are exactly those of calling the
oracle one source after another.  Used where full-size parity needs dozens
of independent solves (64 BFS + 64 SSSP at R-MAT scale 22, 32 BC sources at
scale 23).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def workers() -> int:
    """Threads to use: the host's cores, at most 16 (the CPU share of one GPU)."""
    return max(1, min(16, os.cpu_count() or 1))


def map_sources(fn, sources):
    """[fn(s) for s in sources], the calls spread over worker threads (a line
    is printed as each one finishes: long full-size runs show progress)."""
    sources = list(sources)
    with ThreadPoolExecutor(max_workers=workers()) as ex:
        futs = [ex.submit(fn, int(s)) for s in sources]
        out = []
        for i, f in enumerate(futs):
            out.append(f.result())
            print("[oracle] %d/%d solves done" % (i + 1, len(futs)), flush=True)
        return out


def bfs_rows(row, col, sources):
    return map_sources(lambda s: oracle.bfs(row, col, s), sources)


def sssp_rows(row, col, w, sources):
    return map_sources(lambda s: oracle.sssp(row, col, w, s), sources)


def bc_sum(row, col, sources) -> np.ndarray:
    """FP64 betweenness over `sources`: one oracle call per source, summed in
    source order (the order the oracle's own loop adds them in)."""
    parts = map_sources(lambda s: oracle.bc(row, col, [s]), sources)
    tot = np.zeros(row.size - 1, np.float64)
    for p in parts:
        tot += p
    return tot
