"""CPU oracle for the frontier engine -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``oracle.c``, built with gcc into ``liboracle.so``)
behind a ctypes wrapper.  Only the test-suite, the smoke check and the
benchmark's ``cpu_baseline`` leg may import this package; the product path
(the ``paper_1501_05387_amd`` package and its HIP library) never does, and the
two share no code.

Every function follows a textbook definition named in the paper:

* ``bfs``       hop distance from a source (Sec. 5.1), FIFO-queue BFS.
* ``sssp``      non-negative-weight shortest paths (Sec. 4.1, Sec. 5.2), Dijkstra.
* ``bfs_pred``, ``sssp_pred``  the distances plus a predecessor per vertex (the
  first neighbour in its row one step closer to the source).
* ``bc``        Brandes' two-pass betweenness (Sec. 5.3), FP64.
* ``cc``        component labels (Sec. 5.4), union-find, label = min vertex id.
* ``pagerank``  FP64 power iteration (Sec. 5.5), uniform dangling redistribution.
* ``pagerank_filtered``  the same iteration with per-vertex convergence
  filtering (Sec. 5.5): a vertex leaves the frontier once its rank changes by
  less than a tolerance and keeps that rank from then on.
* ``two_hop``   walks of length two from a seed set (the 2-hop advance, Sec. 4.1).
* ``ppr``       personalized PageRank, teleport and dangling mass to the seeds.
* ``salsa``, ``hits``  bipartite node rankings (hubs left, authorities right),
  the rankings Sec. 5.5 lists as built on the same advance.
* ``advance``, ``advance_edges``, ``filter_ids``  the two operators by their
  definitions, advance from a vertex or from an edge frontier (plain Python,
  for the operator tests).
* ``scan``, ``split``  the exclusive prefix sum and the near/far split of a
  frontier by their definitions (plain Python).

All fifteen are pinned against brute force, closed forms, library routines and
invariants in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SSSP_UNREACHED = np.uint32(0xFFFFFFFF)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Oracle:
    """The oracle bound to one compiled library (the default one, or a test build)."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.or_bfs.restype = i64
        lib.or_bfs.argtypes = [i32, vp, vp, i32, vp]
        lib.or_sssp.restype = i64
        lib.or_sssp.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.or_bc.restype = i32
        lib.or_bc.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.or_cc.restype = i32
        lib.or_cc.argtypes = [i32, vp, vp, vp]
        lib.or_pagerank.restype = i32
        lib.or_pagerank.argtypes = [i32, vp, vp, f64, f64, i32, vp, vp, vp]
        lib.or_pagerank_filtered.restype = i32
        lib.or_pagerank_filtered.argtypes = [i32, vp, vp, f64, f64, i32, vp, vp, vp, vp]
        lib.or_bfs_pred.restype = i64
        lib.or_bfs_pred.argtypes = [i32, vp, vp, i32, vp, vp]
        lib.or_sssp_pred.restype = i64
        lib.or_sssp_pred.argtypes = [i32, vp, vp, vp, i32, vp, vp]
        lib.or_two_hop.restype = i32
        lib.or_two_hop.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.or_ppr.restype = i32
        lib.or_ppr.argtypes = [i32, vp, vp, vp, i32, f64, f64, i32, vp, vp, vp]
        lib.or_salsa.restype = i32
        lib.or_salsa.argtypes = [i32, vp, vp, i32, i32, vp, vp]
        lib.or_hits.restype = i32
        lib.or_hits.argtypes = [i32, vp, vp, i32, i32, vp, vp]
        self.lib = lib
        self.path = libpath

    def bfs(self, row, col, src: int) -> np.ndarray:
        """int32 hop depths from ``src``; unreached vertices get -1."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        depth = np.empty(n, np.int32)
        if self.lib.or_bfs(n, _p(row), _p(col), int(src), _p(depth)) < 0:
            raise ValueError("oracle.bfs: bad input")
        return depth

    def sssp(self, row, col, w, src: int) -> np.ndarray:
        """uint32 shortest distances from ``src``; unreached vertices get 0xFFFFFFFF."""
        row, col, w = _c(row, np.int32), _c(col, np.int32), _c(w, np.uint32)
        n = row.size - 1
        dist = np.empty(n, np.uint32)
        rc = self.lib.or_sssp(n, _p(row), _p(col), _p(w), int(src), _p(dist))
        if rc == -2:
            raise OverflowError("oracle.sssp: a distance does not fit in uint32")
        if rc < 0:
            raise ValueError("oracle.sssp: bad input")
        return dist

    def bfs_pred(self, row, col, src: int):
        """(int32 depths, int32 predecessors): pred[src] = src, -1 unreached, else the first
        neighbour in the row one level up."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        depth, pred = np.empty(n, np.int32), np.empty(n, np.int32)
        if self.lib.or_bfs_pred(n, _p(row), _p(col), int(src), _p(depth), _p(pred)) < 0:
            raise ValueError("oracle.bfs_pred: bad input")
        return depth, pred

    def sssp_pred(self, row, col, w, src: int):
        """(uint32 distances, int32 predecessors): the first neighbour u in the row with
        dist[u] + w = dist[v]."""
        row, col, w = _c(row, np.int32), _c(col, np.int32), _c(w, np.uint32)
        n = row.size - 1
        dist, pred = np.empty(n, np.uint32), np.empty(n, np.int32)
        rc = self.lib.or_sssp_pred(n, _p(row), _p(col), _p(w), int(src), _p(dist), _p(pred))
        if rc == -2:
            raise OverflowError("oracle.sssp_pred: a distance does not fit in uint32")
        if rc < 0:
            raise ValueError("oracle.sssp_pred: bad input")
        return dist, pred

    def bc(self, row, col, sources) -> np.ndarray:
        """FP64 betweenness summed over ``sources`` (unnormalised, ordered pairs)."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        src = _c(sources, np.int32)
        n = row.size - 1
        out = np.empty(n, np.float64)
        if self.lib.or_bc(n, _p(row), _p(col), _p(src), src.size, _p(out)) != 0:
            raise ValueError("oracle.bc: bad input (sources out of range or duplicated)")
        return out

    def cc(self, row, col):
        """(int32 labels = min vertex id per component, number of components)."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        label = np.empty(n, np.int32)
        k = self.lib.or_cc(n, _p(row), _p(col), _p(label))
        if k < 0:
            raise ValueError("oracle.cc: bad input")
        return label, int(k)

    def pagerank(self, row, col, damping: float = 0.85, tol: float = 1e-6, max_iter: int = 1000):
        """(FP64 ranks, iterations run, last L1 change).  ``tol <= 0`` runs exactly max_iter."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        x = np.empty(n, np.float64)
        it = ctypes.c_int32(0)
        l1 = ctypes.c_double(0.0)
        if self.lib.or_pagerank(n, _p(row), _p(col), float(damping), float(tol), int(max_iter),
                                _p(x), ctypes.addressof(it), ctypes.addressof(l1)) != 0:
            raise ValueError("oracle.pagerank: bad input")
        return x, int(it.value), float(l1.value)

    def pagerank_filtered(self, row, col, damping: float, vertex_tol: float, max_iter: int = 1000):
        """(FP64 ranks, iterations run, last summed change, final frontier membership)
        of PageRank with per-vertex convergence filtering."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        x = np.empty(n, np.float64)
        act = np.empty(n, np.uint8)
        it = ctypes.c_int32(0)
        l1 = ctypes.c_double(0.0)
        if self.lib.or_pagerank_filtered(n, _p(row), _p(col), float(damping), float(vertex_tol), int(max_iter),
                                         _p(x), ctypes.addressof(it), ctypes.addressof(l1), _p(act)) != 0:
            raise ValueError("oracle.pagerank_filtered: bad input")
        return x, int(it.value), float(l1.value), act.astype(bool)

    def two_hop(self, row, col, seeds) -> np.ndarray:
        """uint64 number of walks s - u - v of length two from the seed set, per end vertex v."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        sd = _c(seeds, np.int32)
        n = row.size - 1
        out = np.empty(n, np.uint64)
        if self.lib.or_two_hop(n, _p(row), _p(col), _p(sd), sd.size, _p(out)) != 0:
            raise ValueError("oracle.two_hop: bad input (seeds empty, out of range or duplicated)")
        return out

    def ppr(self, row, col, seeds, damping: float = 0.85, tol: float = 1e-9, max_iter: int = 1000):
        """(FP64 personalized PageRank, iterations, last L1 change); teleport uniform over the seeds."""
        row, col = _c(row, np.int32), _c(col, np.int32)
        sd = _c(seeds, np.int32)
        n = row.size - 1
        x = np.empty(n, np.float64)
        it = ctypes.c_int32(0)
        l1 = ctypes.c_double(0.0)
        if self.lib.or_ppr(n, _p(row), _p(col), _p(sd), sd.size, float(damping), float(tol), int(max_iter), _p(x),
                           ctypes.addressof(it), ctypes.addressof(l1)) != 0:
            raise ValueError("oracle.ppr: bad input")
        return x, int(it.value), float(l1.value)

    def _bip(self, fn, name, row, col, n_left: int, iters: int):
        row, col = _c(row, np.int32), _c(col, np.int32)
        n = row.size - 1
        hub = np.empty(max(n_left, 0), np.float64)
        auth = np.empty(max(n - n_left, 0), np.float64)
        if fn(n, _p(row), _p(col), int(n_left), int(iters), _p(hub), _p(auth)) != 0:
            raise ValueError("oracle.%s: bad input (not bipartite across n_left, or bad sizes)" % name)
        return hub, auth

    def salsa(self, row, col, n_left: int, iters: int):
        """(hub scores of [0, n_left), authority scores of [n_left, n)) after `iters` SALSA iterations."""
        return self._bip(self.lib.or_salsa, "salsa", row, col, n_left, iters)

    def hits(self, row, col, n_left: int, iters: int):
        """(unit-L2 hub scores, unit-L2 authority scores) after `iters` HITS iterations."""
        return self._bip(self.lib.or_hits, "hits", row, col, n_left, iters)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else ctypes.addressof(ctypes.c_int64(0))


def bfs(row, col, src: int) -> np.ndarray:
    return default().bfs(row, col, src)


def sssp(row, col, w, src: int) -> np.ndarray:
    return default().sssp(row, col, w, src)


def bc(row, col, sources) -> np.ndarray:
    return default().bc(row, col, sources)


def cc(row, col):
    return default().cc(row, col)


def pagerank(row, col, damping: float = 0.85, tol: float = 1e-6, max_iter: int = 1000):
    return default().pagerank(row, col, damping, tol, max_iter)


def pagerank_filtered(row, col, damping: float, vertex_tol: float, max_iter: int = 1000):
    return default().pagerank_filtered(row, col, damping, vertex_tol, max_iter)


def bfs_pred(row, col, src: int):
    return default().bfs_pred(row, col, src)


def sssp_pred(row, col, w, src: int):
    return default().sssp_pred(row, col, w, src)


def two_hop(row, col, seeds):
    return default().two_hop(row, col, seeds)


def advance(row, col, frontier):
    """The advance operator by its definition (Sec. 4.1): for every frontier entry u in
    order, every edge e of u in CSR order -> arrays (u, e, col[e])."""
    row = np.asarray(row, np.int64)
    src, edge = [], []
    for u in np.asarray(frontier, np.int64).tolist():
        if not 0 <= u < row.size - 1:
            raise ValueError("oracle.advance: vertex out of range")
        e = np.arange(row[u], row[u + 1], dtype=np.int64)
        edge.append(e)
        src.append(np.full(e.size, u, np.int64))
    edge = np.concatenate(edge) if edge else np.zeros(0, np.int64)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    return src.astype(np.int32), edge.astype(np.int32), np.asarray(col, np.int32)[edge]


def advance_edges(row, col, edges):
    """The advance operator from an edge frontier (Sec. 4.1: from edges to their
    neighbouring edges and on to the far-end vertices): for every input edge e in
    order, every edge f of its far end v = col[e] in CSR order -> arrays (e, f, col[f])."""
    row = np.asarray(row, np.int64)
    col = np.asarray(col, np.int64)
    src, edge = [], []
    for e in np.asarray(edges, np.int64).tolist():
        if not 0 <= e < col.size:
            raise ValueError("oracle.advance_edges: edge out of range")
        v = col[e]
        f = np.arange(row[v], row[v + 1], dtype=np.int64)
        edge.append(f)
        src.append(np.full(f.size, e, np.int64))
    edge = np.concatenate(edge) if edge else np.zeros(0, np.int64)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    return src.astype(np.int32), edge.astype(np.int32), col[edge].astype(np.int32)


def scan(values):
    """Exact exclusive prefix sum (the scan that gives the advance its output
    offsets, Sec. 4.4): out[i] = values[0] + ... + values[i-1] as uint64, and the
    total.  numpy's cumulative sum is the step."""
    v = np.asarray(values, np.uint64)
    inc = np.cumsum(v, dtype=np.uint64)
    out = np.zeros(v.size, np.uint64)
    out[1:] = inc[:-1]
    return out, int(inc[-1]) if v.size else 0


def split(items, dist, threshold):
    """The near/far split of a frontier (Sec. 4.5, the priority queue): near =
    the items whose dist is below the threshold, far = the others, each in
    input order."""
    near, far = [], []
    for x in np.asarray(items, np.int64).tolist():
        if not 0 <= x < len(dist):
            raise ValueError("oracle.split: vertex out of range")
        (near if int(dist[x]) < int(threshold) else far).append(x)
    return np.array(near, np.int32), np.array(far, np.int32)


def filter_ids(n, items, exclude=None):
    """The filter operator by its definition (Sec. 4.1): the distinct ids of `items`
    whose exclude byte is 0, ascending."""
    keep = set()
    for v in np.asarray(items, np.int64).tolist():
        if not 0 <= v < n:
            raise ValueError("oracle.filter_ids: vertex out of range")
        if exclude is None or not exclude[v]:
            keep.add(v)
    return np.array(sorted(keep), np.int32)


def ppr(row, col, seeds, damping: float = 0.85, tol: float = 1e-9, max_iter: int = 1000):
    return default().ppr(row, col, seeds, damping, tol, max_iter)


def salsa(row, col, n_left: int, iters: int):
    return default().salsa(row, col, n_left, iters)


def hits(row, col, n_left: int, iters: int):
    return default().hits(row, col, n_left, iters)
