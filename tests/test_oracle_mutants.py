"""The oracle's pins must catch plausible mistakes.

Each case below copies ``oracle/oracle.c``, plants one mistake of the kind a
reader might make (a dropped term, a wrong sign or index, a missing case),
compiles the copy into a temporary library and runs the pins of
``test_oracle_pins.py`` against it.  The test passes only if some pin fails.
The operators' plain-Python definitions get the same treatment: a wrong
version of the function is swapped in for one run of their pins.
The real oracle is never modified.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

ORACLE_C = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, exact source text, replacement)
MUTANTS = [
    ("bfs_depth_from_parent_plus_two", "depth[v] = depth[u] + 1;\n                queue",
     "depth[v] = depth[u] + 2;\n                queue"),
    ("bfs_lifo_instead_of_fifo", "int32_t u = queue[head++];\n        for (int32_t e = R[u]; e < R[u + 1]; ++e) {\n            int32_t v = C[e];\n            if (depth[v] < 0)",
     "int32_t u = queue[--tail];\n        for (int32_t e = R[u]; e < R[u + 1]; ++e) {\n            int32_t v = C[e];\n            if (depth[v] < 0)"),
    ("sssp_ignores_weights", "uint64_t nd = d[u] + (uint64_t)W[e];", "uint64_t nd = d[u] + 1;"),
    ("sssp_weight_of_wrong_edge", "uint64_t nd = d[u] + (uint64_t)W[e];",
     "uint64_t nd = d[u] + (uint64_t)W[R[u]];"),
    ("sssp_heap_sifts_wrong_way", "if (h[p].d <= x.d) break;", "if (h[p].d >= x.d) break;"),
    ("sssp_relax_without_test", "if (nd < d[v]) {\n                d[v] = nd;", "if (1) {\n                d[v] = nd;"),
    ("bc_drops_the_one", "(1.0 + delta[w])", "(delta[w])"),
    ("bc_inverted_ratio", "sigma[v] / sigma[w] *", "sigma[w] / sigma[v] *"),
    ("bc_counts_source", "if (w != s) bc[w] += delta[w];", "bc[w] += delta[w];"),
    ("bc_sigma_from_any_neighbour", "if (depth[v] == depth[u] + 1) sigma[v] += sigma[u];",
     "if (depth[v] != depth[u]) sigma[v] += sigma[u];"),
    ("cc_larger_root_wins", "if (a < b) label[b] = a;\n            else if (b < a) label[a] = b;",
     "if (a < b) label[a] = b;\n            else if (b < a) label[b] = a;"),
    ("cc_no_final_find", "label[v] = uf_find(label, v);\n        if", "(void)0;\n        if"),
    ("pr_drops_dangling", "damping * (s + dangling / N)", "damping * (s)"),
    ("prf_never_filters", "if (dx >= vertex_tol) ++in_frontier;\n            else active[v] = 0;",
     "++in_frontier;"),
    ("prf_strict_threshold", "if (dx >= vertex_tol) ++in_frontier;", "if (dx > vertex_tol) ++in_frontier;"),
    ("prf_frozen_keep_old_value", "x[v] = y[v];\n            if (dx >= vertex_tol) ++in_frontier;\n            else active[v] = 0;",
     "if (dx >= vertex_tol) { ++in_frontier; x[v] = y[v]; }\n            else active[v] = 0;"),
    ("prf_gauss_seidel", "if (active[v]) y[v] = pr_update(", "if (active[v]) x[v] = y[v] = pr_update("),
    ("bfs_pred_last_match", "pred[v] = C[e];\n                break;", "pred[v] = C[e];"),
    ("sssp_pred_any_closer_neighbour", "(uint64_t)dist[u] + W[e] == (uint64_t)dist[v]", "(uint64_t)dist[u] < (uint64_t)dist[v]"),
    ("two_hop_counts_middle_vertex", "for (int32_t f = R[u]; f < R[u + 1]; ++f) count[C[f]] += 1;",
     "for (int32_t f = R[u]; f < R[u + 1]; ++f) count[u] += 1;"),
    ("two_hop_one_hop_only", "for (int32_t f = R[u]; f < R[u + 1]; ++f) count[C[f]] += 1;", "count[u] += 1;"),
    ("ppr_dangling_spread_uniformly", "dangling * p[v]", "dangling / (double)n"),
    ("ppr_teleport_uniform", "(1.0 - damping) * p[v]", "(1.0 - damping) / (double)n"),
    ("salsa_divides_by_target_degree", "s += hub[l] / (double)(R[l + 1] - R[l]);",
     "s += hub[l] / (double)(R[v + 1] - R[v]);"),
    ("salsa_hub_from_unnormalised_auth", "s += auth[v - nl] / (double)(R[v + 1] - R[v]);", "s += auth[v - nl];"),
    ("hits_skips_authority_scaling", "scale_to_unit_l2(auth, nr);", "(void)0;"),
    ("hits_l1_scaling", "for (int32_t i = 0; i < len; ++i) ss += a[i] * a[i];",
     "for (int32_t i = 0; i < len; ++i) ss += fabs(a[i]);"),
    ("pr_teleport_not_divided", "(1.0 - damping) / N + damping", "(1.0 - damping) + damping"),
    ("pr_divides_by_own_degree", "s += x[u] / (double)(R[u + 1] - R[u]);",
     "s += x[u] / (double)(R[v + 1] - R[v]);"),
    ("pr_stops_one_late", "if (tol > 0.0 && l1 < tol) break;", "if (tol > 0.0 && l1 < tol * 0.1) break;"),
]


def _build_mutant(tmp_path, name, old, new):
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, "mutation anchor for %s not unique/absent" % name
    mut = tmp_path / (name + ".c")
    mut.write_text(src.replace(old, new))
    lib = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", str(lib), str(mut), "-lm"])
    return oracle.Oracle(str(lib))


def _all_pins(O):
    pins.pin_exhaustive(O, nmax=5)
    pins.pin_closed_forms(O)
    pins.pin_scipy(O)
    pins.pin_invariants(O)
    pins.pin_pagerank_filtered(O)
    pins.pin_two_hop(O)
    pins.pin_ppr(O)
    pins.pin_salsa(O)
    pins.pin_hits(O)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    O = _build_mutant(tmp_path, name, old, new)
    with pytest.raises((AssertionError, ValueError, OverflowError)):
        _all_pins(O)


# The operator definitions are plain Python (oracle/__init__.py); their mutants
# are wrong versions of the same functions, swapped in for one run of the pins.
_ADVANCE, _ADVANCE_EDGES, _FILTER = oracle.advance, oracle.advance_edges, oracle.filter_ids
_SCAN, _SPLIT = oracle.scan, oracle.split

def _advance_skips_last_edge(row, col, frontier):
    row = np.asarray(row, np.int64)
    src, edge = [], []
    for u in np.asarray(frontier, np.int64).tolist():
        e = np.arange(row[u], max(row[u], row[u + 1] - 1), dtype=np.int64)
        edge.append(e)
        src.append(np.full(e.size, u, np.int64))
    edge = np.concatenate(edge) if edge else np.zeros(0, np.int64)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    return src.astype(np.int32), edge.astype(np.int32), np.asarray(col, np.int32)[edge]


def _advance_sorted_frontier(row, col, frontier):
    return _ADVANCE(row, col, np.sort(np.asarray(frontier, np.int64)))


def _advance_edges_from_tail(row, col, edges):
    row = np.asarray(row, np.int64)
    col = np.asarray(col, np.int64)
    tail = np.repeat(np.arange(row.size - 1), np.diff(row))
    src, edge = [], []
    for e in np.asarray(edges, np.int64).tolist():
        v = tail[e]                                      # the edge's own row instead of its far end
        f = np.arange(row[v], row[v + 1], dtype=np.int64)
        edge.append(f)
        src.append(np.full(f.size, e, np.int64))
    edge = np.concatenate(edge) if edge else np.zeros(0, np.int64)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    return src.astype(np.int32), edge.astype(np.int32), col[edge].astype(np.int32)


def _advance_edges_tags_vertex(row, col, edges):
    src, edge, dst = _ADVANCE_EDGES(row, col, edges)
    return np.asarray(col, np.int32)[src], edge, dst     # tags the far end instead of the input edge


def _filter_keeps_duplicates(n, items, exclude=None):
    keep = [v for v in np.asarray(items, np.int64).tolist() if exclude is None or not exclude[v]]
    return np.array(sorted(keep), np.int32)


def _filter_ignores_exclude(n, items, exclude=None):
    return _FILTER(n, items, None)


def _scan_inclusive(values):
    v = np.asarray(values, np.uint64)
    inc = np.cumsum(v, dtype=np.uint64)
    return inc, int(inc[-1]) if v.size else 0


def _scan_in_32_bits(values):
    out, tot = _SCAN(values)
    return out & np.uint64(0xFFFFFFFF), tot & 0xFFFFFFFF


def _split_at_or_below(items, dist, threshold):
    return _SPLIT(items, dist, int(threshold) + 1)


def _split_far_reversed(items, dist, threshold):
    near, far = _SPLIT(items, dist, threshold)
    return near, far[::-1].copy()


PY_MUTANTS = [
    ("scan_inclusive", "scan", _scan_inclusive),
    ("scan_in_32_bits", "scan", _scan_in_32_bits),
    ("split_at_or_below", "split", _split_at_or_below),
    ("split_far_reversed", "split", _split_far_reversed),
    ("advance_skips_last_edge", "advance", _advance_skips_last_edge),
    ("advance_sorted_frontier", "advance", _advance_sorted_frontier),
    ("advance_edges_from_tail", "advance_edges", _advance_edges_from_tail),
    ("advance_edges_tags_vertex", "advance_edges", _advance_edges_tags_vertex),
    ("filter_keeps_duplicates", "filter_ids", _filter_keeps_duplicates),
    ("filter_ignores_exclude", "filter_ids", _filter_ignores_exclude),
]


@pytest.mark.parametrize("name,attr,fn", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_operator_pins_catch_mutant(monkeypatch, name, attr, fn):
    monkeypatch.setattr(oracle, attr, fn)
    with pytest.raises((AssertionError, ValueError, IndexError)):
        pins.test_operator_definitions()
        pins.test_edge_advance_definition()
        pins.test_scan_definition()
        pins.test_split_definition()
