"""Input generator properties: determinism, symmetric simple CSR, weight symmetry,
source sampling from the largest component."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen


def _check_simple_symmetric(row, col):
    n = row.size - 1
    assert row[0] == 0 and np.all(np.diff(row) >= 0) and row[-1] == col.size
    assert col.size == 0 or (col.min() >= 0 and col.max() < n)
    src = np.repeat(np.arange(n), np.diff(row))
    assert not np.any(src == col), "self loop"
    # strictly increasing inside each row -> sorted, no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # symmetric: the multiset of (u,v) equals the multiset of (v,u)
    key = src.astype(np.int64) * n + col
    rkey = col.astype(np.int64) * n + src
    assert np.array_equal(np.sort(key), np.sort(rkey))


def test_rmat_deterministic_and_simple():
    r1, c1 = graphgen.rmat(12)
    r2, c2 = graphgen.rmat(12)
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    _check_simple_symmetric(r1, c1)
    r3, c3 = graphgen.rmat(12, seed=7)
    assert not (c3.size == c1.size and np.array_equal(c3, c1))
    # no permutation: vertex 0 is the densest corner
    deg = np.diff(r1)
    assert deg[0] == deg.max()


def test_rmat_s16_shape():
    row, col = graphgen.rmat(16)
    assert row.size - 1 == 65536
    assert 1.75e6 < col.size < 1.9e6          # ~1.82M directed entries after dedup
    deg = np.diff(row)
    assert 0.25 < np.mean(deg == 0) < 0.32    # ~28.6 % isolated


def test_grid_shape():
    side = 256
    row, col = graphgen.grid(side)
    _check_simple_symmetric(row, col)
    n = side * side
    nlat = 2 * side * (side - 1)
    und = col.size // 2
    n_long = round(0.001 * nlat)
    assert abs(und - (0.97 * nlat + n_long)) < 5 * np.sqrt(nlat * 0.03 * 0.97) + 2
    assert np.diff(row).max() <= 4 + 8


def test_weights_symmetric_in_range():
    row, col = graphgen.rmat(11)
    w = graphgen.weights(row, col, 64)
    assert w.min() >= 1 and w.max() <= 64
    n = row.size - 1
    M = sp.csr_matrix((w.astype(float), col, row), shape=(n, n))
    assert (M - M.T).nnz == 0
    # roughly uniform over 1..64
    h = np.bincount(w, minlength=65)[1:]
    assert h.min() > 0.5 * h.mean()
    w2 = graphgen.weights(row, col, 1000)
    assert w2.max() <= 1000 and w2.max() > 900


def test_sources_from_largest_component():
    row, col = graphgen.rmat(13)
    n = row.size - 1
    s = graphgen.sample_sources(row, col, 64)
    assert len(set(s.tolist())) == 64
    M = sp.csr_matrix((np.ones(col.size), col, row), shape=(n, n))
    k, lab = csg.connected_components(M, directed=False)
    big = np.argmax(np.bincount(lab))
    assert np.all(lab[s] == big)
    assert np.array_equal(s, graphgen.sample_sources(row, col, 64))


def test_from_edges_drops_loops_and_duplicates():
    row, col = graphgen.from_edges(4, [0, 1, 1, 2, 3], [1, 0, 1, 3, 2])
    assert row.tolist() == [0, 1, 2, 3, 4]
    assert col.tolist() == [1, 0, 3, 2]
