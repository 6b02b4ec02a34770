"""Python binding of the MI355X frontier graph engine (``libgfr.so``).

Argument marshalling only: every step of every solve runs in the HIP library
declared in ``include/gfr.h``.  PyTorch provides device buffers and streams;
results are returned as torch tensors on the context's device unless a
caller-owned ``out`` tensor (device) or numpy array (host) is given.

There is no fallback: if the compiled library is missing, importing a
function that needs it raises ``ImportError`` -- build it with
``python -m paper_1501_05387_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfr.so")
# tuning file written by ``python -m paper_1501_05387_amd.autotune`` on an MI355X
# (R-MAT s16/s20/s22 for the scale-free class, a 2048^2 lattice for the mesh class)
TUNED_PATH = os.path.join(_HERE, "tuning_mi355x.json")


def tuned_json() -> str:
    """The packaged MI355X tuning file (for ``Context(tuning_json=...)``)."""
    with open(TUNED_PATH) as f:
        return f.read()

GFR_OK, GFR_E_INVALID, GFR_E_OOM, GFR_E_DEVICE = 0, -1, -2, -3
GFR_E_NOT_FOUND, GFR_E_NOT_READY, GFR_E_CAPACITY = -4, -5, -6
GFR_VALIDATE = 1
GFR_Q_BFS, GFR_Q_SSSP = 1, 2
STATUS_NAMES = {0: "GFR_OK", -1: "GFR_E_INVALID", -2: "GFR_E_OOM", -3: "GFR_E_DEVICE",
                -4: "GFR_E_NOT_FOUND", -5: "GFR_E_NOT_READY", -6: "GFR_E_CAPACITY"}

# every symbol declared in include/gfr.h: (name, restype, argtypes)
_vp, _i32, _i64, _u32, _u64, _f32, _f64, _cp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float,
                                                 ctypes.c_double, ctypes.c_char_p)


class Query(ctypes.Structure):
    """Mirror of ``gfr_query``."""
    _fields_ = [("kind", _i32), ("source", _i32), ("graph", _i64), ("out", _vp),
                ("out_on_device", _i32), ("reserved", _i32), ("user_tag", _u64)]


SIGNATURES = {
    "gfr_ctx_create": (_i32, [_i32, _cp, ctypes.POINTER(_vp)]),
    "gfr_ctx_destroy": (_i32, [_vp]),
    "gfr_last_error": (_cp, [_vp]),
    "gfr_set_option": (_i32, [_vp, _cp, _f64]),
    "gfr_get_option": (_i32, [_vp, _cp, ctypes.POINTER(_f64)]),
    "gfr_get_stat": (_i32, [_vp, _cp, ctypes.POINTER(_f64)]),
    "gfr_validate_csr": (_i32, [_i32, _i64, _vp, _vp, _vp, _u32, _cp, _i32]),
    "gfr_graph_load_csr": (_i32, [_vp, _i32, _i64, _vp, _vp, _vp, _u32, ctypes.POINTER(_i64)]),
    "gfr_graph_free": (_i32, [_vp, _i64]),
    "gfr_graph_info": (_i32, [_vp, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_u64)]),
    "gfr_bfs": (_i32, [_vp, _i64, _i32, _vp, _vp, _vp]),
    "gfr_bfs_noalloc": (_i32, [_vp, _i64, _i32, _vp, _vp]),
    "gfr_sssp": (_i32, [_vp, _i64, _i32, _vp, _vp, _vp]),
    "gfr_bc": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp]),
    "gfr_cc": (_i32, [_vp, _i64, _vp, ctypes.POINTER(_i32), _vp]),
    "gfr_pagerank": (_i32, [_vp, _i64, _f32, _f64, _i32, _vp, ctypes.POINTER(_i32),
                            ctypes.POINTER(_f64), _vp]),
    "gfr_pagerank_filtered": (_i32, [_vp, _i64, _f64, _f64, _i32, _vp, _vp, ctypes.POINTER(_i32),
                                     ctypes.POINTER(_f64), _vp]),
    "gfr_advance": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp]),
    "gfr_advance_edges": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp]),
    "gfr_scan": (_i32, [_vp, _vp, _i64, _vp, ctypes.POINTER(_u64), _vp]),
    "gfr_split": (_i32, [_vp, _i64, _vp, _i64, _vp, _u32, _vp, _vp, _i64, ctypes.POINTER(_i64),
                         ctypes.POINTER(_i64), _vp]),
    "gfr_filter": (_i32, [_vp, _i64, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp]),
    "gfr_two_hop": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp]),
    "gfr_ppr": (_i32, [_vp, _i64, _vp, _i32, _f64, _f64, _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_f64),
                       _vp]),
    "gfr_salsa": (_i32, [_vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "gfr_hits": (_i32, [_vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "gfr_bfs_batch": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp]),
    "gfr_sssp_batch": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp]),
    "gfr_submit_queries": (_i32, [_vp, ctypes.POINTER(Query), _i32, ctypes.POINTER(_i64)]),
    "gfr_poll": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i32), _i32]),
    "gfr_cancel": (_i32, [_vp, _i64]),
}

_lib = None


def lib():
    """Load libgfr.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgfr.so is not built; run `python -m paper_1501_05387_amd.build`")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libgfr.so bind to that one, so both share one runtime
        # (device pointers, streams and the device context).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class GfrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _torch():
    import torch
    return torch


@dataclass
class Graph:
    ctx: "Context"
    handle: int
    n: int
    m: int
    weighted: bool

    def free(self):
        self.ctx._check(lib().gfr_graph_free(self.ctx.ptr, self.handle))


class Context:
    """A gfr_ctx on one HIP device."""

    def __init__(self, device: int = 0, tuning_json: str | None = None):
        self.device = device
        p = _vp()
        st = lib().gfr_ctx_create(device, tuning_json.encode() if tuning_json else None, ctypes.byref(p))
        if st != GFR_OK:
            raise GfrError(st, "gfr_ctx_create failed on device %d" % device)
        self.ptr = p.value

    def close(self):
        if getattr(self, "ptr", None):
            lib().gfr_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- util
    def _check(self, st: int):
        if st != GFR_OK:
            raise GfrError(st, (lib().gfr_last_error(self.ptr) or b"").decode())

    def _stream(self):
        torch = _torch()
        return torch.cuda.current_stream(self.device).cuda_stream

    def _out(self, out, count: int, dtype):
        """(pointer, object to return) for an output of `count` elements."""
        if out is None:
            torch = _torch()
            tdt = {np.int32: torch.int32, np.uint32: torch.int32, np.float32: torch.float32,
                   np.float64: torch.float64, np.uint8: torch.uint8, np.uint64: torch.int64}[dtype]
            t = torch.empty(count, dtype=tdt, device="cuda:%d" % self.device)
            return t.data_ptr(), t
        if isinstance(out, np.ndarray):
            if out.dtype != np.dtype(dtype) or out.size != count or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous %s array of %d elements" % (np.dtype(dtype), count))
            return out.ctypes.data, out
        # torch tensor
        size = np.dtype(dtype).itemsize
        if out.numel() != count or not out.is_contiguous() or out.element_size() != size:
            raise ValueError("out must be a contiguous %d-byte tensor of %d elements" % (size, count))
        return out.data_ptr(), out

    def set_option(self, key: str, value: float):
        self._check(lib().gfr_set_option(self.ptr, key.encode(), float(value)))

    def get_option(self, key: str) -> float:
        v = _f64()
        self._check(lib().gfr_get_option(self.ptr, key.encode(), ctypes.byref(v)))
        return v.value

    def stat(self, key: str) -> float:
        v = _f64()
        self._check(lib().gfr_get_stat(self.ptr, key.encode(), ctypes.byref(v)))
        return v.value

    # -------------------------------------------------------------- graphs
    def graph_load_csr(self, row, col, weights=None, validate: bool = False) -> Graph:
        row = _np(row, np.int32)
        col = _np(col, np.int32)
        n = row.size - 1
        w = _np(weights, np.uint32) if weights is not None else None
        h = _i64()
        colp = col.ctypes.data if col.size else None
        wp = w.ctypes.data if (w is not None and w.size) else (None if w is None else ctypes.addressof(_u32(0)))
        self._check(lib().gfr_graph_load_csr(self.ptr, n, col.size, row.ctypes.data, colp, wp,
                                             GFR_VALIDATE if validate else 0, ctypes.byref(h)))
        return Graph(self, h.value, n, int(col.size), w is not None)

    def graph_info(self, g: Graph):
        n, m, b = _i32(), _i64(), _u64()
        self._check(lib().gfr_graph_info(self.ptr, g.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(b)))
        return n.value, m.value, b.value

    # ---------------------------------------------------------- primitives
    def _pred(self, pred, n):
        """(pointer or None, object to return or None) for an optional predecessor output."""
        if pred is None or pred is False:
            return None, None
        return self._out(None if pred is True else pred, n, np.int32)

    def bfs(self, g: Graph, source: int, out=None, pred=None):
        """Depths; with pred=True (or a buffer) also the predecessors: (depth, pred)."""
        p, ret = self._out(out, g.n, np.int32)
        pp, pret = self._pred(pred, g.n)
        self._check(lib().gfr_bfs(self.ptr, g.handle, int(source), p, pp, self._stream()))
        return ret if pret is None else (ret, pret)

    def bfs_noalloc(self, g: Graph, source: int, out):
        """Depths into `out` (a device tensor of n int32 the caller allocated)
        through the entry point that allocates nothing."""
        if out is None:
            raise ValueError("bfs_noalloc writes into a caller-allocated device tensor")
        p, ret = self._out(out, g.n, np.int32)
        self._check(lib().gfr_bfs_noalloc(self.ptr, g.handle, int(source), p, self._stream()))
        return ret

    def sssp(self, g: Graph, source: int, out=None, pred=None):
        """Distances; with pred=True (or a buffer) also the predecessors: (dist, pred)."""
        p, ret = self._out(out, g.n, np.uint32)
        pp, pret = self._pred(pred, g.n)
        self._check(lib().gfr_sssp(self.ptr, g.handle, int(source), p, pp, self._stream()))
        return ret if pret is None else (ret, pret)

    def bc(self, g: Graph, sources, out=None):
        src = _np(sources, np.int32)
        p, ret = self._out(out, g.n, np.float32)
        self._check(lib().gfr_bc(self.ptr, g.handle, src.ctypes.data, src.size, p, self._stream()))
        return ret

    def cc(self, g: Graph, out=None):
        p, ret = self._out(out, g.n, np.int32)
        k = _i32()
        self._check(lib().gfr_cc(self.ptr, g.handle, p, ctypes.byref(k), self._stream()))
        return ret, k.value

    def pagerank(self, g: Graph, damping: float = 0.85, tol: float = 1e-6, max_iter: int = 1000, out=None):
        p, ret = self._out(out, g.n, np.float32)
        it, l1 = _i32(), _f64()
        self._check(lib().gfr_pagerank(self.ptr, g.handle, float(damping), float(tol), int(max_iter), p,
                                       ctypes.byref(it), ctypes.byref(l1), self._stream()))
        return ret, it.value, l1.value

    def pagerank_filtered(self, g: Graph, damping: float = 0.85, vertex_tol: float = 1e-9,
                          max_iter: int = 1000, out=None, active=None):
        """(FP64 ranks, final frontier bytes, iterations, last summed change)."""
        p, ret = self._out(out, g.n, np.float64)
        pa, act = self._out(active, g.n, np.uint8)
        it, l1 = _i32(), _f64()
        self._check(lib().gfr_pagerank_filtered(self.ptr, g.handle, float(damping), float(vertex_tol),
                                                int(max_iter), p, pa, ctypes.byref(it), ctypes.byref(l1),
                                                self._stream()))
        return ret, act, it.value, l1.value

    def advance(self, g: Graph, frontier, out_cap=None):
        """Edge frontier of a vertex frontier (numpy array or device tensor of int32 ids):
        (src, edge, dst) device tensors, in frontier order then CSR order."""
        return self._advance("gfr_advance", g, frontier, out_cap)

    def advance_edges(self, g: Graph, edges, out_cap=None):
        """Advance from an edge frontier (int32 edge ids): for every input edge e, every
        edge f of its far end, as (e, f, C[f]) device tensors, in input order then CSR order."""
        return self._advance("gfr_advance_edges", g, edges, out_cap)

    def _advance(self, name, g, frontier, out_cap):
        call = getattr(lib(), name)
        torch = _torch()
        dev = "cuda:%d" % self.device
        if isinstance(frontier, torch.Tensor):
            fr = frontier.to(dev, torch.int32).contiguous()
            fp, nf = fr.data_ptr(), fr.numel()
        else:
            fr = _np(frontier, np.int32)
            fp, nf = (fr.ctypes.data if fr.size else None), fr.size
        cnt = _i64()
        if out_cap is None:   # size the outputs from a counting call
            st = call(self.ptr, g.handle, fp, nf, None, None, None, 0, ctypes.byref(cnt), self._stream())
            if st not in (GFR_OK, GFR_E_CAPACITY):
                self._check(st)
            out_cap = cnt.value
        outs = [torch.empty(max(int(out_cap), 1), dtype=torch.int32, device=dev) for _ in range(3)]
        self._check(call(self.ptr, g.handle, fp, nf, outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr(),
                         int(out_cap), ctypes.byref(cnt), self._stream()))
        k = cnt.value
        return outs[0][:k], outs[1][:k], outs[2][:k]

    def filter(self, g: Graph, items, exclude=None):
        """Ascending distinct ids of `items` whose exclude byte is 0 (device int32 tensor)."""
        torch = _torch()
        dev = "cuda:%d" % self.device
        if isinstance(items, torch.Tensor):
            it = items.to(dev, torch.int32).contiguous()
            ip, cnt_in = it.data_ptr(), it.numel()
        else:
            it = _np(items, np.int32)
            ip, cnt_in = (it.ctypes.data if it.size else None), it.size
        ep = None
        if exclude is not None:
            if isinstance(exclude, torch.Tensor):
                ex = exclude.to(dev, torch.uint8).contiguous()
                ep = ex.data_ptr()
            else:
                ex = _np(exclude, np.uint8)
                ep = ex.ctypes.data
        cap = min(cnt_in, g.n)
        out = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        cnt = _i64()
        self._check(lib().gfr_filter(self.ptr, g.handle, ip, cnt_in, ep, out.data_ptr(), cap, ctypes.byref(cnt),
                                     self._stream()))
        return out[:cnt.value]

    def _list_arg(self, x, np_dtype):
        """(pointer, count, keep-alive) of 32-bit values: a numpy array (converted to
        np_dtype) or a tensor moved to this device (32-bit tensors are passed as they are)."""
        torch = _torch()
        if isinstance(x, torch.Tensor):
            t = x.to("cuda:%d" % self.device)
            if t.dtype not in (torch.int32, torch.uint32):
                t = t.to(torch.int32)
            t = t.contiguous()
            return t.data_ptr(), t.numel(), t
        a = _np(x, np_dtype)
        return (a.ctypes.data if a.size else None), a.size, a

    def scan(self, values):
        """Exclusive prefix sum of uint32 values (numpy array or tensor): (uint64 sums as an
        int64 device tensor, total)."""
        torch = _torch()
        vp, cnt_in, keep = self._list_arg(values, np.uint32)
        out = torch.empty(max(cnt_in, 1), dtype=torch.int64, device="cuda:%d" % self.device)
        tot = _u64()
        self._check(lib().gfr_scan(self.ptr, vp, cnt_in, out.data_ptr(), ctypes.byref(tot), self._stream()))
        del keep
        return out[:cnt_in], tot.value

    def split(self, g: Graph, items, dist, threshold):
        """Near/far split of `items` by dist[v] < threshold (dist: n uint32 values, numpy or
        tensor): (near, far) int32 device tensors, each in input order."""
        torch = _torch()
        ip, cnt_in, keep_i = self._list_arg(items, np.int32)
        dp, nd, keep_d = self._list_arg(dist, np.uint32)
        if nd != g.n:
            raise ValueError("split: dist must hold n = %d values" % g.n)
        cap = max(cnt_in, 1)
        outs = [torch.empty(cap, dtype=torch.int32, device="cuda:%d" % self.device) for _ in range(2)]
        nn, nf = _i64(), _i64()
        self._check(lib().gfr_split(self.ptr, g.handle, ip, cnt_in, dp, int(threshold), outs[0].data_ptr(),
                                    outs[1].data_ptr(), cap, ctypes.byref(nn), ctypes.byref(nf), self._stream()))
        del keep_i, keep_d
        return outs[0][:nn.value], outs[1][:nf.value]

    def two_hop(self, g: Graph, seeds, out=None):
        """Walks of length two from the seed set, per end vertex (int64 tensor or uint64 array)."""
        sd = _np(seeds, np.int32)
        p, ret = self._out(out, g.n, np.uint64)
        self._check(lib().gfr_two_hop(self.ptr, g.handle, sd.ctypes.data, sd.size, p, self._stream()))
        return ret

    def ppr(self, g: Graph, seeds, damping: float = 0.85, tol: float = 1e-9, max_iter: int = 1000, out=None):
        """(FP64 personalized PageRank, iterations, last L1 change)."""
        sd = _np(seeds, np.int32)
        p, ret = self._out(out, g.n, np.float64)
        it, l1 = _i32(), _f64()
        self._check(lib().gfr_ppr(self.ptr, g.handle, sd.ctypes.data, sd.size, float(damping), float(tol),
                                  int(max_iter), p, ctypes.byref(it), ctypes.byref(l1), self._stream()))
        return ret, it.value, l1.value

    def _bipartite(self, fn, g: Graph, n_left: int, iters: int, hub, auth):
        ph, rh = self._out(hub, n_left, np.float64)
        pa, ra = self._out(auth, g.n - n_left, np.float64)
        self._check(fn(self.ptr, g.handle, int(n_left), int(iters), ph, pa, self._stream()))
        return rh, ra

    def salsa(self, g: Graph, n_left: int, iters: int, hub=None, auth=None):
        """(hub scores of [0, n_left), authority scores of [n_left, n)) after `iters` SALSA iterations."""
        return self._bipartite(lib().gfr_salsa, g, n_left, iters, hub, auth)

    def hits(self, g: Graph, n_left: int, iters: int, hub=None, auth=None):
        """(unit-L2 hub scores, unit-L2 authority scores) after `iters` HITS iterations."""
        return self._bipartite(lib().gfr_hits, g, n_left, iters, hub, auth)

    def bfs_batch(self, g: Graph, sources, out=None):
        src = _np(sources, np.int32)
        p, ret = self._out(out, g.n * src.size, np.int32)
        self._check(lib().gfr_bfs_batch(self.ptr, g.handle, src.ctypes.data, src.size, p, self._stream()))
        return ret

    def sssp_batch(self, g: Graph, sources, out=None):
        src = _np(sources, np.int32)
        p, ret = self._out(out, g.n * src.size, np.uint32)
        self._check(lib().gfr_sssp_batch(self.ptr, g.handle, src.ctypes.data, src.size, p, self._stream()))
        return ret

    # ------------------------------------------------------------- serving
    def submit_queries(self, queries):
        """queries: list of (kind, graph, source, out) with `out` a device tensor or host array."""
        arr = (Query * len(queries))()
        for i, (kind, g, src, out) in enumerate(queries):
            on_dev = not isinstance(out, np.ndarray)
            ptr = out.data_ptr() if on_dev else out.ctypes.data
            arr[i] = Query(kind, int(src), g.handle, ptr, 1 if on_dev else 0, 0, i)
        tickets = (_i64 * len(queries))()
        self._check(lib().gfr_submit_queries(self.ptr, arr, len(queries), tickets))
        return list(tickets)

    def poll(self, cap: int = 64, timeout_us: int = 0):
        done = (_i64 * cap)()
        stat = (_i32 * cap)()
        nd = _i32()
        self._check(lib().gfr_poll(self.ptr, done, stat, cap, ctypes.byref(nd), int(timeout_us)))
        return [(done[i], stat[i]) for i in range(nd.value)]

    def cancel(self, ticket: int):
        self._check(lib().gfr_cancel(self.ptr, int(ticket)))


def validate_csr(row, col, weights=None, validate: bool = True):
    """Host-only CSR check (no device needed).  Returns (ok, reason)."""
    row = _np(row, np.int32)
    col = _np(col, np.int32)
    w = _np(weights, np.uint32) if weights is not None else None
    buf = ctypes.create_string_buffer(512)
    st = lib().gfr_validate_csr(row.size - 1, col.size, row.ctypes.data, col.ctypes.data if col.size else None,
                                w.ctypes.data if (w is not None and w.size) else None,
                                GFR_VALIDATE if validate else 0, buf, 512)
    return st == GFR_OK, buf.value.decode()
