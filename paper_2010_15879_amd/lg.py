"""Python binding of liblg (include/lg.h): argument marshalling only.

Every step of encoding, decoding, BFS and PageRank runs in the HIP kernels of
liblg.so; PyTorch provides device memory and the current HIP stream.  If the
library is not built this module raises on import of the library -- there is
no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblg.so")

# -- constants of include/lg.h --------------------------------------------
LG_OK, LG_ERR_INVALID, LG_ERR_OOM, LG_ERR_DEVICE, LG_ERR_UNSUPPORTED, LG_ERR_CAPACITY = range(6)
# limits of lg_decode_neighbors_noalloc (include/lg.h)
LG_NOALLOC_MAX_VERTICES = 65536
LG_NOALLOC_MAX_SORTED_IDS = 1 << 20
STATUS_NAMES = {0: "LG_OK", 1: "LG_ERR_INVALID", 2: "LG_ERR_OOM", 3: "LG_ERR_DEVICE",
                4: "LG_ERR_UNSUPPORTED", 5: "LG_ERR_CAPACITY"}
LAYOUTS = {"packed": 0, "plain": 1}
ID_MODES = {"global": 0, "local": 1, "local-gap": 2, "varint-full": 3, "varint-diff": 4}
OFFSET_MODES = {"packed": 0, "succinct": 1, "ef": 1, "plain-bv": 2, "interleaved-bv": 3}
DECODE_FLAGS = {"sorted": 0, "original": 1, "raw": 2}
BFS_FLAGS = {"do": 0, "direction-opt": 0, "top-down": 1, "td": 1, "bottom-up": 2, "bu": 2}
EXPORTS = {"adj": 0, "offsets": 1, "widths": 2, "ef_low": 3, "ef_high": 4, "ef_rank": 5,
           "ef_select": 6, "perm": 7, "inv": 8, "gap_widths": 9, "weights": 10, "bv_interleaved": 11}
_EXPORT_DTYPE = {"ef_rank": np.uint32, "ef_select": np.uint32, "perm": np.uint32, "inv": np.uint32,
                 "weights": np.uint32}


class LGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class EncodeOpts(C.Structure):
    _fields_ = [("layout", C.c_uint32), ("id_mode", C.c_uint32), ("offset_mode", C.c_uint32),
                ("relabel", C.c_uint32), ("flags", C.c_uint32), ("reserved", C.c_uint32 * 3)]


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_uint64), ("m", C.c_uint64), ("layout", C.c_uint32), ("id_mode", C.c_uint32),
                ("offset_mode", C.c_uint32), ("relabel", C.c_uint32), ("s", C.c_uint32), ("F", C.c_uint32),
                ("w_offset", C.c_uint32), ("ef_l", C.c_uint32), ("universe", C.c_uint64),
                ("adj_bits", C.c_uint64), ("ef_high_bits", C.c_uint64), ("bytes_adj", C.c_uint64),
                ("bytes_offsets", C.c_uint64), ("bytes_widths", C.c_uint64), ("bytes_perm", C.c_uint64),
                ("device_bytes", C.c_uint64), ("max_degree", C.c_uint32), ("isolated", C.c_uint32),
                ("heavy_threshold", C.c_uint32), ("n_heavy", C.c_uint32), ("n_segments", C.c_uint64),
                ("heavy_edges", C.c_uint64), ("heavy_bits", C.c_uint64), ("weight_bits", C.c_uint32),
                ("reserved_w", C.c_uint32), ("bytes_weights", C.c_uint64)]


class BfsJob(C.Structure):
    _fields_ = [("graph", C.c_uint32), ("root", C.c_uint32), ("out_offset", C.c_uint64)]


class BatchInfo(C.Structure):
    _fields_ = [("num_jobs", C.c_uint32), ("workgroups", C.c_uint32), ("threads", C.c_uint32),
                ("chunk", C.c_uint32), ("wave_threshold", C.c_uint32), ("candidates", C.c_uint32),
                ("tuned_ms", C.c_double), ("scratch_bytes", C.c_uint64)]


class ServerOpts(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("workers", C.c_uint32), ("max_batch", C.c_uint32),
                ("reserved", C.c_uint32 * 4)]


class Query(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("graph", C.c_uint32), ("vertex", C.c_uint32), ("k", C.c_int32),
                ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class QueryResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("kind", C.c_uint32), ("count", C.c_uint64),
                ("ids", C.POINTER(C.c_uint32)), ("depth", C.POINTER(C.c_int32)), ("parent", C.POINTER(C.c_int32)),
                ("n", C.c_uint64), ("max_depth", C.c_int32), ("batch", C.c_uint32), ("digest", C.c_uint64),
                ("queue_ms", C.c_double), ("service_ms", C.c_double), ("latency_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("queued", C.c_uint64), ("running", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("resident_bytes", C.c_uint64), ("in_use_bytes", C.c_uint64), ("peak_bytes", C.c_uint64),
                ("workers", C.c_uint32), ("overruns", C.c_uint32), ("batches", C.c_uint64)]


QUERY_KINDS = {"neighbors": 0, "khop": 1, "bfs": 2}

_lib = None

FUNCTIONS = {
    "lg_encode": (C.c_int, [C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p, C.POINTER(EncodeOpts), C.c_void_p,
                            C.POINTER(C.c_void_p)]),
    "lg_decode_neighbors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_uint64,
                                      C.c_uint32, C.c_void_p]),
    "lg_decode_neighbors_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                              C.c_uint64, C.c_uint32, C.c_void_p]),
    "lg_bfs": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.c_uint32, C.c_void_p, C.c_void_p, C.c_int32,
                         C.c_uint32, C.c_void_p]),
    "lg_pagerank": (C.c_int, [C.c_void_p, C.c_float, C.c_uint32, C.c_void_p, C.c_void_p]),
    "lg_encode_weighted": (C.c_int, [C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(EncodeOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "lg_sssp": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]),
    "lg_free": (None, [C.c_void_p]),
    "lg_info": (C.c_int, [C.c_void_p, C.POINTER(GraphInfo)]),
    "lg_export": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint64]),
    "lg_export_bytes": (C.c_uint64, [C.c_void_p, C.c_uint32]),
    "lg_last_error": (C.c_char_p, []),
    "lg_trim": (None, []),
    "lg_prof_enable": (C.c_int, [C.c_int]),
    "lg_prof_filter": (C.c_int, [C.c_char_p]),
    "lg_prof_reset": (C.c_int, []),
    "lg_prof_query": (C.c_int, [C.c_char_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]),
    "lg_prof_names": (C.c_int, [C.c_char_p, C.c_uint64]),
    "lg_bfs_batch_plan": (C.c_int, [C.POINTER(C.c_void_p), C.c_uint32, C.POINTER(BfsJob), C.c_uint32, C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lg_bfs_batch_run": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lg_bfs_batch_info": (C.c_int, [C.c_void_p, C.POINTER(BatchInfo)]),
    "lg_bfs_batch_free": (None, [C.c_void_p]),
    "lg_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_uint32, C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]),
    "lg_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Query), C.POINTER(C.c_uint64)]),
    "lg_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(QueryResult)]),
    "lg_server_result": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(QueryResult)]),
    "lg_server_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.c_uint32, C.POINTER(C.c_uint32)]),
    "lg_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "lg_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "lg_server_free": (None, [C.c_void_p]),
    "lg_admission_simulate": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                        C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]),
}


def lib() -> C.CDLL:
    """Load liblg.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                          f"python paper_2010_15879_amd/build.py")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in FUNCTIONS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != LG_OK:
        msg = lib().lg_last_error()
        raise LGError(status, msg.decode() if msg else "")


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_ptr(t: Optional[torch.Tensor], dtype, what: str) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


class Graph:
    """A representation built by lg_encode; owns the device arrays."""

    def __init__(self, handle: int, n: int, m: int):
        self._h = C.c_void_p(handle)
        self.n = n
        self.m = m

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise ValueError("graph already freed")
        return self._h

    def free(self):
        if self._h:
            lib().lg_free(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        out = GraphInfo()
        _check(lib().lg_info(self.handle, C.byref(out)))
        return {k: getattr(out, k) for k, _ in GraphInfo._fields_}

    def export(self, which: str) -> np.ndarray:
        code = EXPORTS[which]
        nbytes = int(lib().lg_export_bytes(self.handle, code))
        inf = self.info()
        if which == "adj" and inf["layout"] == LAYOUTS["plain"]:
            dtype = np.uint32
        elif which == "offsets" and inf["layout"] == LAYOUTS["plain"]:
            dtype = np.uint64 if inf["m"] >= (1 << 32) else np.uint32
        else:
            dtype = _EXPORT_DTYPE.get(which, np.uint64)
        buf = np.zeros(nbytes // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib().lg_export(self.handle, code, buf.ctypes.data_as(C.c_void_p), nbytes))
        return buf


def _weights_u32(w: torch.Tensor) -> torch.Tensor:
    """The weights as the uint32 bit patterns lg_encode_weighted reads (in an
    int32 tensor), after checking that every value lies in [0, 2^32)."""
    if not w.is_cuda:
        raise ValueError("weights must be a device tensor")
    if w.numel() == 0:
        return w.to(torch.int32)
    if w.dtype == torch.uint32:
        return w.contiguous().view(torch.int32)
    if w.dtype not in (torch.int32, torch.int64):
        raise ValueError(f"weights must be int64, int32 or uint32, got {w.dtype}")
    lo, hi = int(w.min()), int(w.max())
    if lo < 0 or hi >= 1 << 32:
        raise ValueError(f"weights must lie in [0, 2^32), got [{lo}, {hi}]")
    if w.dtype == torch.int32:
        return w.contiguous()
    # values in [2^31, 2^32) become the int32 with the same low 32 bits
    return torch.where(w >= 1 << 31, w - (1 << 32), w).to(torch.int32).contiguous()


def encode(row_offsets: torch.Tensor, col: torch.Tensor, n: Optional[int] = None, *, layout="packed",
           ids="global", offsets="packed", relabel=False, weights: Optional[torch.Tensor] = None,
           stream=None) -> Graph:
    """lg_encode over a device CSR (row_offsets int64[n+1], col int32[M]).
    relabel: False, True or "degree" (degree-minimizing), or "greedy" (the
    greedy heuristic).  weights (a device tensor of M values in [0, 2^32):
    int64, int32 with no negative value, or uint32): an edge weight per
    entry, passed to lg_encode_weighted as uint32."""
    n = row_offsets.numel() - 1 if n is None else n
    m = col.numel()
    if relabel is True or relabel == "degree":
        rl = 1
    elif relabel == "greedy":
        rl = 2
    elif relabel is False or relabel is None:
        rl = 0
    else:
        raise ValueError(f"relabel must be False, True, 'degree' or 'greedy', not {relabel!r}")
    opts = EncodeOpts(LAYOUTS[layout], ID_MODES[ids], OFFSET_MODES[offsets], rl, 0)
    out = C.c_void_p()
    if weights is not None:
        if weights.numel() != m:
            raise ValueError("weights must hold one value per entry of col")
        weights = _weights_u32(weights)
        _check(lib().lg_encode_weighted(n, m, _dev_ptr(row_offsets, torch.int64, "row_offsets"),
                                        _dev_ptr(col, torch.int32, "col") if m else None,
                                        _dev_ptr(weights, torch.int32, "weights") if m else None, C.byref(opts),
                                        _stream(stream), C.byref(out)))
        return Graph(out.value, n, m)
    _check(lib().lg_encode(n, m, _dev_ptr(row_offsets, torch.int64, "row_offsets"),
                           _dev_ptr(col, torch.int32, "col") if m else None, C.byref(opts), _stream(stream),
                           C.byref(out)))
    return Graph(out.value, n, m)


def sssp(g: Graph, root: int, delta: int = 0, stream=None) -> torch.Tensor:
    """lg_sssp: int64[n] distances from root (-1 where not reached)."""
    dist = torch.empty(g.n, dtype=torch.int64, device=torch.device("cuda", torch.cuda.current_device()))
    _check(lib().lg_sssp(g.handle, int(root), int(delta), C.c_void_p(dist.data_ptr()), _stream(stream)))
    return dist


def decode_neighbors(g: Graph, vertices: torch.Tensor, flags="sorted", cap: Optional[int] = None, stream=None):
    """Returns (offsets int64[k+1], ids int32[total]) on the device."""
    k = vertices.numel()
    dev = vertices.device
    off = torch.empty(k + 1, dtype=torch.int64, device=dev)
    vptr = _dev_ptr(vertices, torch.int32, "vertices") if k else None
    s = _stream(stream)
    if cap is None:
        st = lib().lg_decode_neighbors(g.handle, vptr, k, off.data_ptr(), None, 0, DECODE_FLAGS[flags], s)
        if st not in (LG_OK, LG_ERR_CAPACITY):
            _check(st)
        cap = int(off[-1].item())
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    _check(lib().lg_decode_neighbors(g.handle, vptr, k, off.data_ptr(), ids.data_ptr(), cap, DECODE_FLAGS[flags], s))
    return off, ids[: int(off[-1].item())]


def decode_neighbors_noalloc(g: Graph, vertices: torch.Tensor, out_off: torch.Tensor, out_ids: torch.Tensor,
                             flags="sorted", stream=None) -> int:
    """lg_decode_neighbors_noalloc into caller-provided device tensors
    (out_off int64[k+1], out_ids int32[cap]); returns the lg_status (LG_OK or
    LG_ERR_CAPACITY) and raises on every other status."""
    k = vertices.numel()
    if out_off.numel() != k + 1:
        raise ValueError("out_off must hold k + 1 entries")
    vptr = _dev_ptr(vertices, torch.int32, "vertices") if k else None
    st = lib().lg_decode_neighbors_noalloc(g.handle, vptr, k, _dev_ptr(out_off, torch.int64, "out_off"),
                                           _dev_ptr(out_ids, torch.int32, "out_ids") if out_ids.numel() else None,
                                           out_ids.numel(), DECODE_FLAGS[flags], _stream(stream))
    if st not in (LG_OK, LG_ERR_CAPACITY):
        _check(st)
    return st


def bfs(g: Graph, roots: Sequence[int], *, parent=True, max_depth=-1, mode="do", depth_out=None,
        parent_out=None, stream=None):
    """Returns (depth int32[r, n], parent int32[r, n] or None)."""
    r = len(roots)
    dev = torch.device("cuda", torch.cuda.current_device())
    depth = depth_out if depth_out is not None else torch.empty((r, g.n), dtype=torch.int32, device=dev)
    par = parent_out if parent_out is not None else (
        torch.empty((r, g.n), dtype=torch.int32, device=dev) if parent else None)
    for t, what in [(depth, "depth"), (par, "parent")]:
        if t is not None and t.numel() < r * g.n:
            raise ValueError(f"{what} must hold {r} x {g.n} entries, got {t.numel()}")
    arr = (C.c_uint32 * max(r, 1))(*[int(x) for x in roots])
    _check(lib().lg_bfs(g.handle, arr, r, _dev_ptr(depth, torch.int32, "depth"),
                        _dev_ptr(par, torch.int32, "parent"), max_depth, BFS_FLAGS[mode], _stream(stream)))
    return depth, par


def pagerank(g: Graph, damping: float = 0.85, iters: int = 20, out=None, stream=None) -> torch.Tensor:
    dev = torch.device("cuda", torch.cuda.current_device())
    scores = out if out is not None else torch.empty(g.n, dtype=torch.float32, device=dev)
    if scores.numel() < g.n:
        raise ValueError(f"out must hold {g.n} entries, got {scores.numel()}")
    _check(lib().lg_pagerank(g.handle, float(damping), int(iters), _dev_ptr(scores, torch.float32, "scores"),
                             _stream(stream)))
    return scores


# -- kernel timing ------------------------------------------------------

def prof_enable(on: bool = True):
    _check(lib().lg_prof_enable(1 if on else 0))


def prof_filter(substr: str = ""):
    _check(lib().lg_prof_filter(substr.encode()))


def prof_reset():
    _check(lib().lg_prof_reset())


def prof_query(kernel: str):
    launches = C.c_uint64()
    ms = C.c_double()
    _check(lib().lg_prof_query(kernel.encode(), C.byref(launches), C.byref(ms)))
    return int(launches.value), float(ms.value)


def prof_names() -> list:
    buf = C.create_string_buffer(1 << 16)
    lib().lg_prof_names(buf, len(buf))
    return [x for x in buf.value.decode().split("\n") if x]


# -- batched BFS -----------------------------------------------------------

class BatchPlan:
    """A captured persistent launch running many BFS queries (lg_bfs_batch_*).

    jobs: list of (graph index, root).  Results: depth[i] / parent[i] are the
    rows of query i (views into flat device buffers)."""

    def __init__(self, graphs, jobs, *, parent=True, max_depth=-1, autotune=True, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.graphs = list(graphs)
        self.jobs = list(jobs)
        # a bad graph index is left for the library to reject (LG_ERR_INVALID)
        sizes = [self.graphs[g].n if 0 <= g < len(self.graphs) else 0 for g, _ in self.jobs]
        offs = [0]
        for s_ in sizes:
            offs.append(offs[-1] + s_)
        self.offsets = offs
        self.depth_flat = torch.empty(max(offs[-1], 1), dtype=torch.int32, device=dev)
        self.parent_flat = torch.empty(max(offs[-1], 1), dtype=torch.int32, device=dev) if parent else None
        arr_g = (C.c_void_p * len(self.graphs))(*[g.handle.value for g in self.graphs])
        arr_j = (BfsJob * max(len(self.jobs), 1))(*[BfsJob(g, r, offs[i]) for i, (g, r) in enumerate(self.jobs)])
        out = C.c_void_p()
        _check(lib().lg_bfs_batch_plan(arr_g, len(self.graphs), arr_j, len(self.jobs), self.depth_flat.data_ptr(),
                                       self.parent_flat.data_ptr() if parent else None, max_depth,
                                       1 if autotune else 0, _stream(stream), C.byref(out)))
        self._p = out

    def run(self, stream=None):
        _check(lib().lg_bfs_batch_run(self._p, _stream(stream)))

    def info(self) -> dict:
        out = BatchInfo()
        _check(lib().lg_bfs_batch_info(self._p, C.byref(out)))
        return {k: getattr(out, k) for k, _ in BatchInfo._fields_}

    def depth(self, i):
        return self.depth_flat[self.offsets[i]:self.offsets[i + 1]]

    def parent(self, i):
        return self.parent_flat[self.offsets[i]:self.offsets[i + 1]]

    def free(self):
        if self._p:
            lib().lg_bfs_batch_free(self._p)
            self._p = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# -- query server -----------------------------------------------------------

class Server:
    """lg_server_*: queries over resident graphs, served by worker threads with
    their own streams, admitted under a device-memory budget."""

    def __init__(self, graphs, budget_bytes=0, workers=8, max_batch=64):
        self.graphs = list(graphs)
        arr = (C.c_void_p * len(self.graphs))(*[g.handle.value for g in self.graphs])
        opts = ServerOpts(int(budget_bytes), int(workers), int(max_batch))
        out = C.c_void_p()
        _check(lib().lg_server_create(arr, len(self.graphs), C.byref(opts), C.byref(out)))
        self._s = out

    def submit(self, kind, graph, vertex, k=0, keep_arrays=False) -> int:
        q = Query(QUERY_KINDS[kind], graph, vertex, k, 1 if keep_arrays else 0, 0)
        t = C.c_uint64()
        _check(lib().lg_server_submit(self._s, C.byref(q), C.byref(t)))
        return int(t.value)

    @staticmethod
    def _unpack(r: QueryResult, arrays=True) -> dict:
        out = {k: getattr(r, k) for k, _ in QueryResult._fields_ if k not in ("ids", "depth", "parent")}
        if not arrays:
            return out
        out["ids"] = np.ctypeslib.as_array(r.ids, shape=(r.count,)).copy() if r.ids else np.zeros(0, np.uint32)
        if r.depth:
            out["depth"] = np.ctypeslib.as_array(r.depth, shape=(r.n,)).copy()
            out["parent"] = np.ctypeslib.as_array(r.parent, shape=(r.n,)).copy()
        return out

    def wait(self, ticket: int, release=True, arrays=True) -> dict:
        """Block until the query completes; arrays=False skips copying the
        returned IDs / BFS arrays into numpy."""
        r = QueryResult()
        _check(lib().lg_server_wait(self._s, ticket, C.byref(r)))
        out = self._unpack(r, arrays)
        if release:
            lib().lg_server_release(self._s, ticket)
        return out

    def poll(self, cap=4096) -> list:
        arr = (C.c_uint64 * cap)()
        cnt = C.c_uint32()
        _check(lib().lg_server_poll(self._s, arr, cap, C.byref(cnt)))
        return [int(arr[i]) for i in range(cnt.value)]

    def result(self, ticket: int, release=True) -> dict:
        r = QueryResult()
        _check(lib().lg_server_result(self._s, ticket, C.byref(r)))
        out = self._unpack(r)
        if release:
            lib().lg_server_release(self._s, ticket)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().lg_server_get_stats(self._s, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def free(self):
        if self._s:
            lib().lg_server_free(self._s)
            self._s = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def admission_simulate(arrival, need, service, budget, resident, workers):
    """Host-only model of the server's admission (lg_admission_simulate)."""
    n = len(arrival)
    a = (C.c_double * max(n, 1))(*arrival)
    nd = (C.c_uint64 * max(n, 1))(*[int(x) for x in need])
    sv = (C.c_double * max(n, 1))(*service)
    st = (C.c_double * max(n, 1))()
    fi = (C.c_double * max(n, 1))()
    ss = (C.c_int32 * max(n, 1))()
    pk = C.c_uint64()
    _check(lib().lg_admission_simulate(a, nd, sv, n, int(budget), int(resident), int(workers), st, fi, ss,
                                       C.byref(pk)))
    return list(st)[:n], list(fi)[:n], list(ss)[:n], int(pk.value)


def trim():
    """Free the device buffers lg_encode keeps for reuse (lg_trim)."""
    lib().lg_trim()
