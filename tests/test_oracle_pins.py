"""Pins for the CPU oracle: every check here comes from somewhere other than the
oracle itself -- brute force on tiny graphs, closed forms, scipy's graph
routines, dense linear algebra and invariants that any correct answer obeys.

The pins are written as functions of an oracle object so that
``test_oracle_mutants.py`` can run them against deliberately broken builds of
the oracle and show that each plausible mistake is caught.
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen
import oracle
from tests import brute
from tests import invariants as inv


# --------------------------------------------------------------- helpers ----
def _csr_matrix(row, col, data=None):
    n = row.size - 1
    if data is None:
        data = np.ones(col.size)
    return sp.csr_matrix((np.asarray(data, float), col, row), shape=(n, n))


def _path(n):
    return graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n))


def _star(n):
    return graphgen.from_edges(n, np.zeros(n - 1, np.int32), np.arange(1, n))


def _complete(n):
    iu = np.triu_indices(n, 1)
    return graphgen.from_edges(n, iu[0], iu[1])


def _lattice(side):
    """Undropped side x side lattice (no long edges), built from an explicit edge list."""
    eu, ev = [], []
    for r in range(side):
        for c in range(side):
            v = r * side + c
            if c + 1 < side:
                eu.append(v); ev.append(v + 1)
            if r + 1 < side:
                eu.append(v); ev.append(v + side)
    return graphgen.from_edges(side * side, eu, ev)


# ------------------------------------------------------ exhaustive pins ----
def pin_exhaustive(O, nmax=5, seed=0):
    """All labelled simple graphs on 1..nmax vertices vs Floyd-Warshall,
    walk-count path numbers, Freeman BC and a dense PageRank solve."""
    rng = np.random.default_rng(seed)
    for n in range(1, nmax + 1):
        for A in brute.all_simple_graphs(n):
            row, col, _ = brute.csr_from_adj(A)
            D = brute.floyd_warshall(A)
            # BFS from every source = unit-weight shortest hop counts
            for s in range(n):
                want = np.where(np.isfinite(D[s]), D[s], -1).astype(np.int32)
                got = O.bfs(row, col, s)
                assert np.array_equal(got, want), (n, A.tolist(), s)
            # SSSP with random symmetric weights
            Wm = np.triu(rng.integers(1, 10, size=(n, n)), 1)
            Wm = (Wm + Wm.T) * A
            rowW, colW, wW = brute.csr_from_adj(Wm)
            DW = brute.floyd_warshall(Wm)
            for s in range(n):
                want = np.where(np.isfinite(DW[s]), DW[s], 0xFFFFFFFF).astype(np.uint32)
                assert np.array_equal(O.sssp(rowW, colW, wW, s), want), (n, Wm.tolist(), s)
            # predecessors: the smallest neighbour one step closer (rows are sorted)
            for s in range(n):
                dep, pred = O.bfs_pred(row, col, s)
                _, predw = O.sssp_pred(rowW, colW, wW, s)
                for v in range(n):
                    if not np.isfinite(D[s][v]):
                        assert pred[v] == -1 and predw[v] == -1
                        continue
                    if v == s:
                        assert pred[v] == s and predw[v] == s
                        continue
                    up = [u for u in range(n) if A[u, v] and D[s][u] == D[s][v] - 1]
                    assert pred[v] == min(up), (A.tolist(), s, v)
                    upw = [u for u in range(n) if Wm[u, v] and DW[s][u] + Wm[u, v] == DW[s][v]]
                    assert predw[v] == min(upw), (Wm.tolist(), s, v)
            # CC labels = smallest reachable id
            lab, k = O.cc(row, col)
            want = brute.component_min_labels(D)
            assert np.array_equal(lab, want)
            assert k == len(set(want.tolist()))
            # BC over all sources and over a random subset
            assert np.allclose(O.bc(row, col, np.arange(n)), brute.freeman_bc(A, range(n)),
                               rtol=1e-12, atol=1e-12)
            S = rng.permutation(n)[: max(1, n // 2)]
            assert np.allclose(O.bc(row, col, S), brute.freeman_bc(A, S), rtol=1e-12, atol=1e-12)
            # PageRank to a tight tolerance vs the fixed point
            x, it, l1 = O.pagerank(row, col, 0.85, 1e-15, 10000)
            assert np.allclose(x, brute.pagerank_solve(A, 0.85), rtol=0, atol=1e-13)


def test_exhaustive_small_graphs(orc):
    pin_exhaustive(orc)


# -------------------------------------------------------- closed forms ----
def pin_closed_forms(O):
    n = 33
    row, col = _path(n)
    for s in (0, 7, n - 1):
        assert np.array_equal(O.bfs(row, col, s), np.abs(np.arange(n) - s))
    i = np.arange(n)
    assert np.allclose(O.bc(row, col, np.arange(n)), 2.0 * i * (n - 1 - i))

    row, col = _star(n)
    d = O.bfs(row, col, 0)
    assert d[0] == 0 and np.all(d[1:] == 1)
    bcv = O.bc(row, col, np.arange(n))
    assert bcv[0] == (n - 1) * (n - 2) and np.all(bcv[1:] == 0)
    # star K_{1,k}: the centre c and each leaf l satisfy
    #   c = (1-d)/N + d*k*l,   l = (1-d)/N + d*c/k
    k = n - 1
    dd = 0.85
    A2 = np.array([[1.0, -dd * k], [-dd / k, 1.0]])
    c_, l_ = np.linalg.solve(A2, [(1 - dd) / n, (1 - dd) / n])
    x, _, _ = O.pagerank(row, col, dd, 1e-15, 10000)
    assert abs(x[0] - c_) < 1e-14 and np.allclose(x[1:], l_, atol=1e-14)

    row, col = _complete(9)
    assert np.all(O.bc(row, col, np.arange(9)) == 0)
    x, _, _ = O.pagerank(row, col, 0.85, 1e-15, 10000)
    assert np.allclose(x, 1.0 / 9, atol=1e-15)          # regular graph

    side = 17
    row, col = _lattice(side)
    rr, cc = np.divmod(np.arange(side * side), side)
    for s in (0, 5 * side + 9):
        man = np.abs(rr - rr[s]) + np.abs(cc - cc[s])
        assert np.array_equal(O.bfs(row, col, s), man)
        w1 = np.ones(col.size, np.uint32)
        assert np.array_equal(O.sssp(row, col, w1, s), man.astype(np.uint32))
        w3 = np.full(col.size, 3, np.uint32)
        assert np.array_equal(O.sssp(row, col, w3, s), 3 * man.astype(np.uint32))
    lab, k = O.cc(row, col)
    assert k == 1 and np.all(lab == 0)


def test_closed_forms(orc):
    pin_closed_forms(orc)


# ------------------------------------------------- scipy cross-checks ----
def _random_graph(rng, n, p):
    A = np.triu(rng.random((n, n)) < p, 1)
    iu = np.nonzero(A)
    return graphgen.from_edges(n, iu[0], iu[1])


def pin_scipy(O, seed=1):
    rng = np.random.default_rng(seed)
    cases = [_random_graph(rng, n, p) for n, p in ((50, 0.05), (120, 0.02), (200, 0.01), (200, 0.04))]
    cases.append(graphgen.rmat(10, 8, seed=5))
    for row, col in cases:
        n = row.size - 1
        w = graphgen.weights(row, col, 64, seed=9)
        M1 = _csr_matrix(row, col)
        MW = _csr_matrix(row, col, w)
        srcs = rng.choice(n, size=4, replace=False)
        Dh = csg.shortest_path(M1, directed=False, unweighted=True, indices=srcs)
        Dw = csg.dijkstra(MW, directed=False, indices=srcs)
        for i, s in enumerate(srcs):
            want = np.where(np.isfinite(Dh[i]), Dh[i], -1).astype(np.int32)
            assert np.array_equal(O.bfs(row, col, s), want)
            want = np.where(np.isfinite(Dw[i]), Dw[i], 0xFFFFFFFF).astype(np.uint32)
            assert np.array_equal(O.sssp(row, col, w, s), want)
        k_sp, lab_sp = csg.connected_components(M1, directed=False)
        lab, k = O.cc(row, col)
        assert k == k_sp
        # same partition, and each label is the minimum id of its part
        mins = np.full(k_sp, n, np.int64)
        np.minimum.at(mins, lab_sp, np.arange(n))
        assert np.array_equal(lab, mins[lab_sp])


def test_scipy_crosscheck(orc):
    pin_scipy(orc)


# --------------------------------------------- invariants at mid size ----
def pin_invariants(O):
    row, col = graphgen.rmat(14)
    n = row.size - 1
    w = graphgen.weights(row, col, 64)
    srcs = graphgen.sample_sources(row, col, 4)
    depths = []
    for s in srcs:
        d = O.bfs(row, col, s)
        inv.check_bfs(row, col, s, d)
        depths.append(d)
        dist = O.sssp(row, col, w, s)
        inv.check_sssp(row, col, w, s, dist)
        assert np.array_equal(dist != 0xFFFFFFFF, d >= 0)
        # unit weights turn SSSP into BFS
        assert np.array_equal(O.sssp(row, col, np.ones_like(w), s).astype(np.int64),
                              np.where(d >= 0, d.astype(np.int64), 0xFFFFFFFF))
        # predecessor trees: a neighbour one step closer, and every chain ends at the source
        dep, pred = O.bfs_pred(row, col, s)
        dist2, predw = O.sssp_pred(row, col, w, s)
        assert np.array_equal(dep, d) and np.array_equal(dist2, dist)
        for p_, key in ((pred, d.astype(np.int64)), (predw, np.where(dist == 0xFFFFFFFF, -1, dist.astype(np.int64)))):
            reached = key >= 0
            assert np.array_equal(p_ >= 0, reached) and p_[s] == s
            v = np.nonzero(reached & (np.arange(n) != s))[0]
            u = p_[v]
            assert np.all(key[u] < key[v])            # strictly closer (weights >= 1)
            nb = set(zip(np.repeat(np.arange(n), np.diff(row)).tolist(), col.tolist()))
            assert all((int(a), int(b)) in nb for a, b in zip(v[:2000], u[:2000]))
    lab, k = O.cc(row, col)
    assert inv.check_cc(row, col, lab) == k
    bcv = O.bc(row, col, srcs)
    assert np.all(bcv >= 0)
    ident = inv.bc_pair_identity(depths)
    assert abs(bcv.sum() - ident) <= 1e-9 * max(1.0, ident)
    x, it, l1 = O.pagerank(row, col, 0.85, 1e-6, 1000)
    assert abs(x.sum() - 1.0) < 1e-12 and np.all(x > 0)
    assert l1 < 1e-6
    # contraction: ||x_k - x*|| <= d/(1-d) ||x_k - x_{k-1}||
    xs, _, _ = O.pagerank(row, col, 0.85, 1e-15, 10000)
    assert np.abs(x - xs).sum() <= 0.85 / 0.15 * l1 * (1 + 1e-9)
    # running exactly k-1 then k iterations reproduces the reported L1 change
    xa, ka, l1a = O.pagerank(row, col, 0.85, 0.0, it - 1)
    assert l1a >= 1e-6, "the stop rule must fire at the first iteration below tol"
    xb, kb, l1b = O.pagerank(row, col, 0.85, 0.0, it)
    assert ka == it - 1 and kb == it
    assert np.array_equal(xb, x) and abs(np.abs(xb - xa).sum() - l1) < 1e-18


def test_invariants_rmat(orc):
    pin_invariants(orc)


# ------------------------------- PageRank with convergence filtering ----
def _star_iso_classes(k, n_iso, d, eps, max_iter):
    """Filtered PageRank on a star K_{1,k} plus n_iso isolated vertices,
    reduced by symmetry to three classes (centre, leaves, isolated): every
    member of a class has the same value and leaves the frontier in the same
    iteration.  Returns (values, iterations, last change, still active, the
    smallest distance between a change and eps over all decisions)."""
    N = 1 + k + n_iso
    val = {"c": 1.0 / N, "l": 1.0 / N, "i": 1.0 / N}
    cnt = {"c": 1, "l": k, "i": n_iso}
    act = {"c": True, "l": True, "i": n_iso > 0}
    if n_iso == 0:
        del val["i"], cnt["i"], act["i"]
    it, l1, margin = 0, 0.0, np.inf
    while it < max_iter and any(act.values()):
        D = n_iso * val.get("i", 0.0)
        new = {"c": (1 - d) / N + d * (k * val["l"] + D / N),
               "l": (1 - d) / N + d * (val["c"] / k + D / N),
               "i": (1 - d) / N + d * (D / N)}
        l1 = 0.0
        for cl in val:
            if act[cl]:
                dx = abs(new[cl] - val[cl])
                l1 += cnt[cl] * dx
                val[cl] = new[cl]
                margin = min(margin, abs(dx - eps))
                act[cl] = dx >= eps
        it += 1
    return val, it, l1, act, margin


def pin_pagerank_filtered(O):
    # tolerance 0 never shrinks the frontier: identical to plain power iteration
    for row, col in (graphgen.rmat(10, 8, seed=3), graphgen.from_edges(7, [0, 1, 2], [1, 2, 0])):
        for iters in (1, 6, 25):
            x, it, l1, act = O.pagerank_filtered(row, col, 0.85, 0.0, iters)
            xp, itp, l1p = O.pagerank(row, col, 0.85, 0.0, iters)
            assert it == iters == itp and np.array_equal(x, xp) and l1 == l1p and act.all()
    # a change of exactly zero stays in the frontier at tolerance 0: K_2 with
    # d = 1/2 is at its fixed point (1/2, 1/2) from the start, exactly
    row, col = _complete(2)
    x, it, l1, act = O.pagerank_filtered(row, col, 0.5, 0.0, 7)
    assert it == 7 and act.all() and l1 == 0.0 and np.all(x == 0.5)
    x, it, l1, act = O.pagerank_filtered(row, col, 0.5, 1e-300, 7)
    assert it == 1 and not act.any()
    # a tolerance above any possible change: one iteration, empty frontier
    row, col = graphgen.rmat(10, 8, seed=3)
    x, it, l1, act = O.pagerank_filtered(row, col, 0.85, 2.0, 50)
    x1, _, l11 = O.pagerank(row, col, 0.85, 0.0, 1)
    assert it == 1 and not act.any() and np.array_equal(x, x1) and l1 == l11
    # a regular graph is at its fixed point: everything leaves at once
    row, col = _complete(9)
    x, it, _, act = O.pagerank_filtered(row, col, 0.85, 1e-12, 50)
    assert it == 1 and not act.any() and np.allclose(x, 1.0 / 9, atol=1e-16)
    # star + isolated vertices against the three-class recurrence; the
    # tolerances make the classes leave the frontier in different iterations
    staggered = False
    for k, n_iso in ((5, 3), (12, 0), (2, 1)):
        g = graphgen.from_edges(1 + k + n_iso, np.zeros(k, np.int32), np.arange(1, k + 1))
        for eps in (1e-3, 3e-5, 1e-7, 1e-10, 1e-13):
            val, it_w, l1_w, act_w, margin = _star_iso_classes(k, n_iso, 0.85, eps, 400)
            assert margin > 1e-6 * eps, "decision too close to eps for a robust pin"
            x, it, l1, act = O.pagerank_filtered(g[0], g[1], 0.85, eps, 400)
            assert it == it_w, (k, n_iso, eps, it, it_w)
            assert abs(x[0] - val["c"]) <= 1e-15 and np.allclose(x[1:k + 1], val["l"], rtol=0, atol=1e-15)
            if n_iso:
                assert np.allclose(x[k + 1:], val["i"], rtol=0, atol=1e-15)
            assert abs(l1 - l1_w) <= 1e-12 * max(l1_w, 1e-300) + 1e-18
            assert act[0] == act_w["c"] and np.all(act[1:k + 1] == act_w["l"])
            if n_iso:
                assert np.all(act[k + 1:] == act_w["i"])
            # the capped run reproduces the classes' state after fewer iterations
            cap = max(1, it_w // 2)
            val2, it2, _, act2, _ = _star_iso_classes(k, n_iso, 0.85, eps, cap)
            x2, it2g, _, a2 = O.pagerank_filtered(g[0], g[1], 0.85, eps, cap)
            assert it2g == it2 and abs(x2[0] - val2["c"]) <= 1e-15 and a2[0] == act2["c"]
            staggered |= n_iso > 0 and len({act2["c"], act2["l"], act2["i"]}) > 1
    assert staggered
    # shrinking the tolerance approaches the fixed point
    row, col = graphgen.rmat(12)
    xs, _, _ = O.pagerank(row, col, 0.85, 1e-15, 10000)
    errs = [np.abs(O.pagerank_filtered(row, col, 0.85, e, 10000)[0] - xs).sum() for e in (1e-6, 1e-9, 1e-13)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-7


def test_pagerank_filtered(orc):
    pin_pagerank_filtered(orc)


# --------------------------------------------- 2-hop and node ranking ----
def _bipartite(rng, nl, nr, p, connect=True):
    """Random bipartite graph, left [0, nl), right [nl, nl + nr); with `connect`
    a spanning path alternating sides keeps it connected."""
    B = rng.random((nl, nr)) < p
    if connect:
        for i in range(max(nl, nr)):
            B[i % nl, i % nr] = True
            B[(i + 1) % nl, i % nr] = True
    l, r = np.nonzero(B)
    row, col = graphgen.from_edges(nl + nr, l, nl + r)
    return row, col, B


def pin_two_hop(O, seed=4):
    rng = np.random.default_rng(seed)
    # every labelled graph on up to 4 vertices, every seed set, against A @ A
    for n in range(1, 5):
        for A in brute.all_simple_graphs(n):
            row, col, _ = brute.csr_from_adj(A)
            A2 = A.astype(np.int64) @ A.astype(np.int64)
            for mask in range(1, 1 << n):
                S = [i for i in range(n) if mask >> i & 1]
                assert np.array_equal(O.two_hop(row, col, S), A2[S].sum(0)), (A.tolist(), S)
    # scipy sparse products on larger graphs; the total is the degree sum of the seeds' neighbours
    for row, col in (_random_graph(rng, 300, 0.02), graphgen.rmat(11), graphgen.grid(40)):
        n = row.size - 1
        M = _csr_matrix(row, col)
        for k in (1, 5, 40):
            S = rng.choice(n, size=k, replace=False)
            want = np.asarray((M[S] @ M).sum(0)).ravel().astype(np.uint64)
            got = O.two_hop(row, col, S)
            assert np.array_equal(got, want)
            deg = np.diff(row)
            assert int(got.sum()) == int(sum(deg[col[row[s]:row[s + 1]]].sum() for s in S))
    row, col = _star(6)
    for bad in ([], [1, 1], [6]):
        with pytest.raises(ValueError):
            O.two_hop(row, col, bad)


def pin_ppr(O, seed=5):
    rng = np.random.default_rng(seed)
    for n in range(1, 6):
        for A in brute.all_simple_graphs(n):
            row, col, _ = brute.csr_from_adj(A)
            S = sorted(rng.choice(n, size=rng.integers(1, n + 1), replace=False).tolist())
            x, it, l1 = O.ppr(row, col, S, 0.85, 1e-15, 10000)
            assert np.allclose(x, brute.ppr_solve(A, 0.85, S), rtol=0, atol=1e-13), (A.tolist(), S)
    row, col = graphgen.rmat(11)
    n = row.size - 1
    # teleport to every vertex is plain PageRank
    x, _, _ = O.ppr(row, col, np.arange(n), 0.85, 1e-14, 10000)
    xp, _, _ = O.pagerank(row, col, 0.85, 1e-14, 10000)
    assert np.abs(x - xp).sum() < 1e-12
    # mass, positivity on the seeds' reach, and the contraction bound
    S = graphgen.sample_sources(row, col, 3)
    x, it, l1 = O.ppr(row, col, S, 0.85, 1e-8, 1000)
    xs, _, _ = O.ppr(row, col, S, 0.85, 1e-15, 10000)
    assert abs(x.sum() - 1.0) < 1e-12 and l1 < 1e-8
    assert np.abs(x - xs).sum() <= 0.85 / 0.15 * l1 * (1 + 1e-9)
    reach = O.bfs(row, col, int(S[0])) >= 0
    assert np.all(xs[reach] > 0) and np.all(xs[~reach] == 0)


def pin_salsa(O, seed=6):
    rng = np.random.default_rng(seed)
    # K_{a,b}: uniform after one iteration
    for a, b in ((1, 1), (3, 5), (7, 2)):
        l, r = np.divmod(np.arange(a * b), b)
        row, col = graphgen.from_edges(a + b, l, a + r)
        h, au = O.salsa(row, col, a, 1)
        assert np.allclose(h, 1.0 / a, atol=1e-16) and np.allclose(au, 1.0 / b, atol=1e-16)
    # connected, no isolated vertex: the scores converge to degree / |E|
    row, col, B = _bipartite(rng, 40, 60, 0.08)
    E = col.size // 2
    deg = np.diff(row).astype(float)
    h, au = O.salsa(row, col, 40, 400)
    assert np.allclose(h, deg[:40] / E, rtol=0, atol=1e-12) and np.allclose(au, deg[40:] / E, rtol=0, atol=1e-12)
    for it in (1, 2, 7):   # the walk keeps its mass
        h, au = O.salsa(row, col, 40, it)
        assert abs(h.sum() - 1) < 1e-12 and abs(au.sum() - 1) < 1e-12
    # two components: each keeps the share of hubs it started with, spread by degree
    r1, c1, _ = _bipartite(rng, 10, 15, 0.2)
    r2, c2, _ = _bipartite(rng, 30, 20, 0.1)
    s1 = np.repeat(np.arange(25), np.diff(r1))
    s2 = np.repeat(np.arange(50), np.diff(r2))
    relabel1 = np.where(np.arange(25) < 10, np.arange(25), 40 + (np.arange(25) - 10))
    relabel2 = np.where(np.arange(50) < 30, 10 + np.arange(50), 40 + 15 + (np.arange(50) - 30))
    eu = np.concatenate([relabel1[s1], relabel2[s2]])
    ev = np.concatenate([relabel1[c1], relabel2[c2]])
    row, col = graphgen.from_edges(75, eu, ev)
    deg = np.diff(row).astype(float)
    h, au = O.salsa(row, col, 40, 600)
    E1, E2 = c1.size // 2, c2.size // 2
    want_h = np.concatenate([10 / 40 * deg[:10] / E1, 30 / 40 * deg[10:40] / E2])
    want_a = np.concatenate([10 / 40 * deg[40:55] / E1, 30 / 40 * deg[55:] / E2])
    assert np.allclose(h, want_h, rtol=0, atol=1e-12) and np.allclose(au, want_a, rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        O.salsa(*_path(4), 1, 3)      # edge 1-2 stays inside the right side


def pin_hits(O, seed=7):
    rng = np.random.default_rng(seed)
    for a, b in ((1, 1), (3, 5), (7, 2)):
        l, r = np.divmod(np.arange(a * b), b)
        row, col = graphgen.from_edges(a + b, l, a + r)
        h, au = O.hits(row, col, a, 1)
        assert np.allclose(h, 1 / np.sqrt(a), atol=1e-15) and np.allclose(au, 1 / np.sqrt(b), atol=1e-15)
    row, col, B = _bipartite(rng, 50, 35, 0.1)
    U, sv, Vt = np.linalg.svd(B.astype(float))
    u1, v1 = np.abs(U[:, 0]), np.abs(Vt[0])
    assert sv[0] - sv[1] > 0.1 * sv[0]           # a clear gap, so the iteration converges fast
    h, au = O.hits(row, col, 50, 300)
    assert np.allclose(h, u1, rtol=0, atol=1e-10) and np.allclose(au, v1, rtol=0, atol=1e-10)
    for it in (1, 3):
        h, au = O.hits(row, col, 50, it)
        assert abs(np.linalg.norm(h) - 1) < 1e-14 and abs(np.linalg.norm(au) - 1) < 1e-14


def test_two_hop(orc):
    pin_two_hop(orc)


def test_ppr(orc):
    pin_ppr(orc)


def test_salsa(orc):
    pin_salsa(orc)


def test_hits(orc):
    pin_hits(orc)


def test_input_validation(orc):
    row, col = _path(5)
    with pytest.raises(ValueError):
        orc.bfs(row, col, 5)
    with pytest.raises(ValueError):
        orc.bc(row, col, [1, 1])
    with pytest.raises(ValueError):
        orc.pagerank(row, col, 1.0)
    w = np.full(col.size, 0x7FFFFFFF, np.uint32)
    with pytest.raises(OverflowError):
        orc.sssp(row, col, w, 0)


# ------------------------------------------------------------ operators ----
def test_operator_definitions():
    """The advance and filter oracles: a worked example, then agreement with the
    adjacency matrix (rows of a sorted CSR list neighbours in ascending order)."""
    row, col = _path(5)                                  # 0-1-2-3-4
    src, edge, dst = oracle.advance(row, col, [1, 1, 4, 0])
    assert src.tolist() == [1, 1, 1, 1, 4, 0]
    assert dst.tolist() == [0, 2, 0, 2, 3, 1]
    assert np.array_equal(col[edge], dst)
    assert oracle.filter_ids(5, [4, 1, 1, 3, 0], [0, 0, 0, 1, 0]).tolist() == [0, 1, 4]
    assert oracle.filter_ids(5, []).tolist() == []
    rng = np.random.default_rng(8)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        row, col = _random_graph(rng, n, 0.2)
        A = np.zeros((n, n), bool)
        A[np.repeat(np.arange(n), np.diff(row)), col] = True
        F = rng.integers(0, n, size=int(rng.integers(0, 30)))
        src, edge, dst = oracle.advance(row, col, F)
        want_src = [u for u in F.tolist() for _ in range(int(A[u].sum()))]
        want_dst = [v for u in F.tolist() for v in np.nonzero(A[u])[0].tolist()]
        assert src.tolist() == want_src and dst.tolist() == want_dst
        assert edge.size == int(np.diff(row)[F].sum())
        ex = rng.integers(0, 2, size=n).astype(np.uint8)
        assert oracle.filter_ids(n, F, ex).tolist() == sorted(set(v for v in F.tolist() if not ex[v]))
    with pytest.raises(ValueError):
        oracle.advance(row, col, [n])


def test_edge_advance_definition():
    """advance_edges: a worked example, then the walk counts of the adjacency
    matrix: over every edge (u, v), the pairs (u, far end) it leads to count
    the walks u - v - w, so their histogram is A @ A."""
    row, col = _path(4)                                  # 0-1-2-3; edges 0:0-1 1:1-0 2:1-2 3:2-1 4:2-3 5:3-2
    src, edge, dst = oracle.advance_edges(row, col, [0, 5, 0])
    assert src.tolist() == [0, 0, 5, 5, 0, 0]
    assert edge.tolist() == [1, 2, 3, 4, 1, 2]
    assert dst.tolist() == [0, 2, 1, 3, 0, 2]
    assert [x.size for x in oracle.advance_edges(row, col, [])] == [0, 0, 0]
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        row, col = _random_graph(rng, n, 0.2)
        m = col.size
        A = np.zeros((n, n), np.int64)
        A[np.repeat(np.arange(n), np.diff(row)), col] = 1
        tail = np.repeat(np.arange(n), np.diff(row))     # the row each edge sits in
        src, edge, dst = oracle.advance_edges(row, col, np.arange(m))
        H = np.zeros((n, n), np.int64)
        np.add.at(H, (tail[src], dst), 1)
        assert np.array_equal(H, A @ A)
        E = rng.integers(0, max(m, 1), size=int(rng.integers(0, 30))) if m else np.zeros(0, np.int64)
        src, edge, dst = oracle.advance_edges(row, col, E)
        want_dst = [w for e in E.tolist() for w in np.nonzero(A[col[e]])[0].tolist()]
        assert src.tolist() == [e for e in E.tolist() for _ in range(int(A[col[e]].sum()))]
        assert dst.tolist() == want_dst and np.array_equal(tail[edge], np.repeat(col[E], np.diff(row)[col[E]]))
    with pytest.raises(ValueError):
        oracle.advance_edges(row, col, [col.size])


def test_scan_definition():
    """scan: closed forms (ones give 0..k-1, 0..k-1 give the triangular numbers
    i(i-1)/2, a constant c gives c*i), sums taken one by one on random inputs,
    exactness past 2^32 and 2^53, and the empty input."""
    out, tot = oracle.scan(np.ones(1000, np.uint32))
    assert out.tolist() == list(range(1000)) and tot == 1000
    k = 3000
    out, tot = oracle.scan(np.arange(k, dtype=np.uint32))
    i = np.arange(k, dtype=np.uint64)
    assert np.array_equal(out, i * (i - 1) // 2) and tot == k * (k - 1) // 2
    out, _ = oracle.scan(np.full(500, 7, np.uint32))
    assert np.array_equal(out, 7 * np.arange(500, dtype=np.uint64))
    rng = np.random.default_rng(11)
    for _ in range(10):
        v = rng.integers(0, 2**32, size=int(rng.integers(1, 60)), dtype=np.uint64).astype(np.uint32)
        out, tot = oracle.scan(v)
        acc = 0
        for j, x in enumerate(v.tolist()):
            assert int(out[j]) == acc
            acc += x
        assert tot == acc
    big = np.full(3_000_000, 2**32 - 1, np.uint32)             # total above 2^53
    out, tot = oracle.scan(big)
    assert tot == 3_000_000 * (2**32 - 1) and int(out[-1]) == 2_999_999 * (2**32 - 1)
    out, tot = oracle.scan(np.zeros(0, np.uint32))
    assert out.size == 0 and tot == 0


def test_split_definition():
    """split: a worked example, then on random inputs: near and far together are
    the items (as a multiset), each keeps the input order, every near item is
    below the threshold and every far item is not; thresholds 0 and above every
    value put everything far and near."""
    dist = np.array([5, 0, 9, 3, 3], np.uint32)
    near, far = oracle.split([4, 2, 1, 4, 0, 3], dist, 4)
    assert near.tolist() == [4, 1, 4, 3] and far.tolist() == [2, 0]
    rng = np.random.default_rng(12)
    for _ in range(20):
        n = int(rng.integers(1, 50))
        d = rng.integers(0, 100, size=n).astype(np.uint32)
        X = rng.integers(0, n, size=int(rng.integers(0, 80)))
        t = int(rng.integers(0, 110))
        near, far = oracle.split(X, d, t)
        assert sorted(near.tolist() + far.tolist()) == sorted(X.tolist())
        assert np.all(d[near] < t) and np.all(d[far] >= t)
        assert near.tolist() == [x for x in X.tolist() if d[x] < t]
        assert far.tolist() == [x for x in X.tolist() if d[x] >= t]
        assert oracle.split(X, d, 0)[0].size == 0
        assert oracle.split(X, d, 101)[1].size == 0
    with pytest.raises(ValueError):
        oracle.split([3], np.zeros(3, np.uint32), 1)
