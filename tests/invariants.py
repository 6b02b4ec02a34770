"""O(m) numpy checks that any correct result must satisfy, at any graph size.

Used to pin the oracle on mid-size graphs and to check GPU results at sizes
where running the oracle for every case would be too slow.
"""
from __future__ import annotations

import numpy as np

UNREACHED32 = np.uint32(0xFFFFFFFF)


def edge_sources(row: np.ndarray) -> np.ndarray:
    n = row.size - 1
    return np.repeat(np.arange(n, dtype=np.int32), np.diff(row))


def check_bfs(row, col, src, depth):
    """depth[src]=0; |d(u)-d(v)| <= 1 on edges; reached set closed; parents exist."""
    n = row.size - 1
    depth = np.asarray(depth)
    assert depth.shape == (n,)
    assert depth[src] == 0
    assert np.all(depth >= -1)
    u = edge_sources(row)
    du, dv = depth[u], depth[col]
    both = (du >= 0) & (dv >= 0)
    assert np.all(np.abs(du[both] - dv[both]) <= 1), "BFS depth jumps by more than one on an edge"
    assert not np.any((du >= 0) ^ (dv >= 0)), "reached set not closed under adjacency"
    # every reached v != src has a neighbour at depth-1
    has_parent = np.zeros(n, bool)
    tight = both & (du == dv - 1)
    has_parent[col[tight]] = True
    need = (depth > 0)
    assert np.all(has_parent[need]), "reached vertex without a parent one level up"


def check_sssp(row, col, w, src, dist):
    """d[src]=0; triangle inequality on every edge; every reached v has a tight edge."""
    n = row.size - 1
    d = np.asarray(dist).astype(np.uint64)
    inf = np.uint64(0xFFFFFFFF)
    assert d[src] == 0
    u = edge_sources(row)
    du, dv = d[u], d[col]
    ww = np.asarray(w).astype(np.uint64)
    reach_u = du != inf
    assert not np.any(reach_u & (dv == inf)), "reached set not closed under adjacency"
    assert np.all(dv[reach_u] <= du[reach_u] + ww[reach_u]), "triangle inequality violated"
    tight = reach_u & (dv == du + ww)
    has = np.zeros(n, bool)
    has[col[tight]] = True
    need = (d != inf) & (np.arange(n) != src)
    assert np.all(has[need]), "reached vertex without a tight incoming edge"


def check_cc(row, col, label):
    """label equal across edges; label[v] <= v; label[label] = label; roots are minima."""
    n = row.size - 1
    lab = np.asarray(label)
    u = edge_sources(row)
    assert np.all(lab[u] == lab[col]), "edge joins two labels"
    assert np.all(lab <= np.arange(n))
    assert np.all(lab[lab] == lab)
    return int(np.sum(lab == np.arange(n)))


def bc_pair_identity(depths_per_source) -> float:
    """sum_v BC_S(v) = sum_{s in S} sum_{t reached, t != s} (d(s,t) - 1)."""
    tot = 0.0
    for dep in depths_per_source:
        r = dep[dep > 0]
        tot += float(np.sum(r - 1))
    return tot
