"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, the binding knows each of them, and the host-only CSR
validation accepts and rejects the right graphs.  No device work here."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import graphgen
import paper_1501_05387_amd as gfr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfr.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gfr_\w+)\s*\(", txt)))


def test_header_declares_the_abi():
    names = header_functions()
    for required in ("gfr_graph_load_csr", "gfr_bfs", "gfr_sssp", "gfr_bc", "gfr_cc", "gfr_pagerank",
                     "gfr_submit_queries", "gfr_poll"):
        assert required in names


def test_library_exports_every_header_symbol():
    L = gfr.lib()
    for name in header_functions():
        assert hasattr(L, name), "libgfr.so does not export %s" % name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_binding_covers_every_header_symbol():
    assert sorted(gfr.SIGNATURES) == header_functions()


def test_library_has_no_oracle_dependency():
    # the product library must not link or embed the oracle
    data = open(gfr.LIB_PATH, "rb").read()
    assert b"or_bfs" not in data and b"liboracle" not in data


def test_package_never_reaches_the_oracle():
    # no module of the product package (nor its kernels' sources) names the oracle
    pkg = os.path.dirname(gfr.__file__)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "or_bfs" not in text, f


def test_binding_fails_loudly_without_the_library():
    # a fresh interpreter pointed at a missing library must raise, not fall back
    code = ("import sys; sys.path.insert(0, %r); import paper_1501_05387_amd as g; "
            "g.LIB_PATH = '/nonexistent/libgfr.so'\n"
            "try:\n    g.Context(0)\nexcept ImportError:\n    sys.exit(0)\nsys.exit(3)") % ROOT
    import subprocess
    import sys
    assert subprocess.run([sys.executable, "-c", code], timeout=300).returncode == 0


def test_validate_accepts_generated_graphs():
    row, col = graphgen.rmat(10)
    w = graphgen.weights(row, col)
    ok, why = gfr.validate_csr(row, col, w)
    assert ok, why
    row, col = graphgen.grid(32)
    assert gfr.validate_csr(row, col)[0]


@pytest.mark.parametrize("case", ["asym", "loop", "dup", "unsorted", "range", "offsets", "wasym"])
def test_validate_rejects(case):
    row = np.array([0, 2, 3, 4], np.int32)
    col = np.array([1, 2, 0, 0], np.int32)
    w = np.array([5, 6, 5, 6], np.uint32)
    assert gfr.validate_csr(row, col, w)[0]
    if case == "asym":
        row, col = np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32)
        w = None
    elif case == "loop":
        row, col, w = np.array([0, 1, 1], np.int32), np.array([0], np.int32), None
    elif case == "dup":
        row, col, w = np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32), None
    elif case == "unsorted":
        row = np.array([0, 2, 3, 4], np.int32)
        col = np.array([2, 1, 0, 0], np.int32)
        w = None
    elif case == "range":
        col = np.array([1, 7, 0, 0], np.int32)
    elif case == "offsets":
        row = np.array([0, 3, 2, 4], np.int32)
    elif case == "wasym":
        w = np.array([5, 6, 5, 7], np.uint32)
    ok, why = gfr.validate_csr(row, col, w)
    assert not ok and why


def test_structural_checks_without_validate_flag():
    row = np.array([0, 1, 1, 1], np.int32)
    col = np.array([1], np.int32)
    assert gfr.validate_csr(row, col, validate=False)[0]          # asymmetric passes the basic check
    assert not gfr.validate_csr(np.array([1, 1], np.int32), np.zeros(0, np.int32), validate=False)[0]


@pytest.mark.parametrize("text,ok", [
    ('{}', True),
    ('{"advance.chunk": 2048, "bfs.alpha": 12.5}', True),
    ('{"scalefree": {"bfs.alpha": 20, "batch.min_sssp": 16}, "mesh": {"sssp.delta": 3000}}', True),
    (' { "mesh" : { } , "serve.max_batch" : 32 } ', True),
    ('{"no.such.option": 1}', False),
    ('{"advance.chunk": 300}', False),                     # not a power of two in range
    ('{"bfs.alpha": -1}', False),                          # out of range
    ('{"mesh": {"serve.max_batch": 8}}', False),          # not a per-class option
    ('{"planar": {"bfs.alpha": 3}}', False),               # unknown class
    ('{"bfs.alpha": "fast"}', False),
    ('{"bfs.alpha": 3', False),
    ('{"bfs.alpha": 3} x', False),
    ('[1, 2]', False),
])
def test_tuning_file_is_checked_before_the_device(text, ok):
    L = gfr.lib()
    p = ctypes.c_void_p()
    st = L.gfr_ctx_create(0, text.encode(), ctypes.byref(p))
    if ok:
        # accepted: fails only for want of a device (or succeeds on a GPU host)
        assert st in (gfr.GFR_OK, gfr.GFR_E_DEVICE), st
        if st == gfr.GFR_OK:
            L.gfr_ctx_destroy(p.value)
    else:
        assert st == gfr.GFR_E_INVALID, st


def test_packaged_tuning_file_is_accepted():
    """The committed MI355X tuning file parses and only holds known options
    (checked before the device is touched)."""
    L = gfr.lib()
    p = ctypes.c_void_p()
    st = L.gfr_ctx_create(0, gfr.tuned_json().encode(), ctypes.byref(p))
    assert st in (gfr.GFR_OK, gfr.GFR_E_DEVICE), st
    if st == gfr.GFR_OK:
        L.gfr_ctx_destroy(p.value)


def test_bench_traffic_digest_covers_existing_sources():
    """The digest that ties a committed HBM-counter figure to the relaxation
    kernel names files that exist and includes every header that kernel's
    source includes, so that an edit to any of them voids the figure."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    pkg = os.path.join(root, "paper_1501_05387_amd")
    for f in bench.RELAX_SOURCES:
        assert os.path.isfile(os.path.join(pkg, f)), f
    src = open(os.path.join(pkg, "csrc", "sssp_batch.hip")).read()
    local = set(re.findall(r'#include "([^"]+)"', src))
    covered = {os.path.basename(f) for f in bench.RELAX_SOURCES}
    for h in local:
        assert os.path.basename(h) in covered, h
    assert len(bench.relax_source_digest()) == 16
    assert bench.relax_source_digest() != bench.kernel_source_digest()


def test_bench_sssp_floor_bytes_counts_each_reached_pair_once():
    """The batched relaxation's algorithmic bytes (the SSSP work model at
    r = 1) equal, summed per query and per reached vertex, 16 B for its
    frontier entry, 12 B per edge leaving it and 8 B for its improvement
    (none for the query's own source), on oracle distances of a small graph
    with an unreachable part."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    import graphgen
    import oracle
    r1, c1 = graphgen.rmat(8)
    n1 = r1.size - 1
    # a second copy of the graph, never reached from sources in the first
    row = np.concatenate([r1, r1[1:] + r1[-1]]).astype(r1.dtype)
    col = np.concatenate([c1, c1 + n1]).astype(c1.dtype)
    w = graphgen.weights(row, col, 64)
    deg = np.diff(row)
    srcs = [0, 3, 3, 17]
    want, pairs, edges = 0, 0, 0
    for s in srcs:
        d = oracle.sssp(row, col, w, s)
        for v in range(row.size - 1):
            if d[v] != 0xFFFFFFFF:
                want += 16 + 12 * int(deg[v]) + (8 if v != s else 0)
        reached = d != 0xFFFFFFFF
        pairs += int(reached.sum())
        edges += int(deg[reached].sum())
    assert pairs < len(srcs) * (row.size - 1)   # the copy stays unreached
    assert bench.bsssp_floor_bytes(pairs, edges, len(srcs)) == want
