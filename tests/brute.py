"""Independent brute-force definitions used to pin the oracle (tiny graphs only).

Nothing here follows the oracle's algorithms: distances come from
Floyd-Warshall, path counts from powers of the adjacency matrix, betweenness
from the pair-dependency (Freeman) definition, PageRank from a dense linear
solve, and components from reachability in the distance matrix.
"""
from __future__ import annotations

import itertools

import numpy as np


def csr_from_adj(A: np.ndarray):
    """Symmetric 0/1 (or weight) matrix -> (row, col, w) CSR with sorted rows."""
    n = A.shape[0]
    row = np.zeros(n + 1, np.int32)
    cols, ws = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols.extend(nz.tolist())
        ws.extend(A[i, nz].tolist())
        row[i + 1] = row[i] + nz.size
    return row, np.asarray(cols, np.int32), np.asarray(ws, np.uint32)


def all_simple_graphs(n: int):
    """Every labelled simple undirected graph on n vertices (2^(n(n-1)/2) of them)."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        A = np.zeros((n, n), np.int64)
        for b, (i, j) in enumerate(pairs):
            if mask >> b & 1:
                A[i, j] = A[j, i] = 1
        yield A


def floyd_warshall(Wm: np.ndarray) -> np.ndarray:
    """All-pairs shortest distances; Wm[i,j] > 0 is an edge weight, 0 means no edge."""
    n = Wm.shape[0]
    D = np.where(Wm > 0, Wm.astype(float), np.inf)
    np.fill_diagonal(D, 0.0)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def path_counts(A: np.ndarray, D: np.ndarray) -> np.ndarray:
    """sigma[s,t] = number of shortest s-t paths = (A^d)[s,t] with d = hop distance.

    A walk of minimum length between two vertices is a path, so counting walks of
    exactly d(s,t) steps counts shortest paths.
    """
    n = A.shape[0]
    sig = np.zeros((n, n))
    P = np.eye(n)
    Af = A.astype(float)
    for d in range(n):
        sig[D == d] = P[D == d]
        P = P @ Af
    return sig


def freeman_bc(A: np.ndarray, sources) -> np.ndarray:
    """BC_S(v) = sum_{s in S} sum_{t != s, t != v} sigma_st(v) / sigma_st, ordered pairs."""
    n = A.shape[0]
    D = floyd_warshall(A)
    sig = path_counts(A, D)
    bc = np.zeros(n)
    for s in sources:
        for t in range(n):
            if t == s or not np.isfinite(D[s, t]):
                continue
            for v in range(n):
                if v in (s, t):
                    continue
                if D[s, v] + D[v, t] == D[s, t]:
                    bc[v] += sig[s, v] * sig[v, t] / sig[s, t]
    return bc


def pagerank_solve(A: np.ndarray, d: float) -> np.ndarray:
    """Fixed point of x = (1-d)/N + d (A^T D^-1 x + (dangling . x)/N) by a dense solve."""
    n = A.shape[0]
    deg = A.sum(1).astype(float)
    M = np.zeros((n, n))
    for u in range(n):
        if deg[u] > 0:
            M[:, u] = A[u, :] / deg[u]
        else:
            M[:, u] = 1.0 / n
    return np.linalg.solve(np.eye(n) - d * M, np.full(n, (1.0 - d) / n))


def ppr_solve(A: np.ndarray, d: float, seeds) -> np.ndarray:
    """Fixed point of x = (1-d) p + d (A^T D^-1 x + (dangling . x) p), p uniform over the
    seeds, by a dense solve."""
    n = A.shape[0]
    p = np.zeros(n)
    p[list(seeds)] = 1.0 / len(seeds)
    deg = A.sum(1).astype(float)
    M = np.zeros((n, n))
    for u in range(n):
        if deg[u] > 0:
            M[:, u] = A[u, :] / deg[u]
        else:
            M[:, u] = p
    return np.linalg.solve(np.eye(n) - d * M, (1.0 - d) * p)


def component_min_labels(D: np.ndarray) -> np.ndarray:
    """label[v] = smallest u reachable from v (finite distance)."""
    n = D.shape[0]
    return np.array([int(np.nonzero(np.isfinite(D[v]))[0].min()) for v in range(n)], np.int32)
