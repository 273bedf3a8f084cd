"""numpy wrappers over the C oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class _NullableU8:
    """ctypes argument type accepting a uint8 array or None."""

    @classmethod
    def from_param(cls, obj):
        if obj is None:
            return None
        return u8p.from_param(obj)


class _NullableU32:
    @classmethod
    def from_param(cls, obj):
        if obj is None:
            return None
        return u32p.from_param(obj)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "lg_oracle.c"))
    ):
        from . import build as _b
        _b.build()
    L = C.CDLL(_LIB_PATH)
    sig = {
        "orc_bitlen": (C.c_uint, [C.c_uint64]),
        "orc_stream_words": (C.c_uint64, [C.c_uint64]),
        "orc_get_bits": (C.c_uint64, [u64p, C.c_uint64, C.c_uint]),
        "orc_global_width": (C.c_uint, [C.c_uint64]),
        "orc_local_widths": (None, [C.c_uint64, u64p, u32p, u8p]),
        "orc_width_field_bits": (C.c_uint, [C.c_uint64]),
        "orc_relabeled_local_widths": (None, [C.c_uint64, u64p, u32p, u32p, u32p, u8p, u64p]),
        "orc_adjacency_bits": (C.c_uint64, [C.c_uint64, u64p, _NullableU8, C.c_uint]),
        "orc_bit_starts": (None, [C.c_uint64, u64p, _NullableU8, C.c_uint, u64p]),
        "orc_pack_adjacency": (None, [C.c_uint64, u64p, u32p, _NullableU8, C.c_uint, u64p]),
        "orc_pack_adjacency_words": (None, [C.c_uint64, u64p, u32p, _NullableU8, C.c_uint,
                                            C.c_uint64, C.c_uint64, u64p]),
        "orc_decode_list": (None, [u64p, C.c_uint64, C.c_uint64, C.c_uint, u32p]),
        "orc_pack_fixed": (None, [u64p, C.c_uint64, C.c_uint, u64p]),
        "orc_rank1": (C.c_uint64, [u64p, C.c_uint64]),
        "orc_select1": (C.c_uint64, [u64p, C.c_uint64, C.c_uint64]),
        "orc_ef_low_bits": (C.c_uint, [C.c_uint64, C.c_uint64]),
        "orc_ef_upper_bits": (C.c_uint64, [C.c_uint64, C.c_uint64, C.c_uint]),
        "orc_ef_rank_entries": (C.c_uint64, [C.c_uint64]),
        "orc_ef_select_entries": (C.c_uint64, [C.c_uint64]),
        "orc_ef_build": (None, [u64p, C.c_uint64, C.c_uint64, u64p, u64p, u32p, u32p]),
        "orc_ef_get": (C.c_uint64, [u64p, u64p, C.c_uint64, C.c_uint, C.c_uint64]),
        "orc_dm_permutation": (None, [C.c_uint64, u64p, u32p, u32p]),
        "orc_relabel": (None, [C.c_uint64, u64p, u32p, u32p, u32p, u64p, u32p]),
        "orc_greedy_permutation": (None, [C.c_uint64, u64p, u32p, u32p, u32p]),
        "orc_gap_widths": (None, [C.c_uint64, u64p, u32p, u8p]),
        "orc_gap_bit_starts": (None, [C.c_uint64, u64p, u8p, u8p, u64p]),
        "orc_pack_gap": (None, [C.c_uint64, u64p, u32p, u8p, u8p, u64p]),
        "orc_decode_gap_list": (None, [u64p, C.c_uint64, C.c_uint64, C.c_uint, C.c_uint, u32p]),
        "orc_varint_len": (C.c_uint, [C.c_uint32]),
        "orc_varint_byte_starts": (None, [C.c_uint64, u64p, u32p, C.c_int, u64p]),
        "orc_pack_varint": (None, [C.c_uint64, u64p, u32p, C.c_int, u8p]),
        "orc_decode_varint_list": (C.c_uint64, [u8p, C.c_uint64, C.c_uint64, C.c_int, u32p]),
        "orc_weight_width": (C.c_uint, [C.c_uint64, u32p]),
        "orc_pack_weighted": (None, [C.c_uint64, u64p, u32p, u32p, _NullableU8, C.c_uint, C.c_uint, u64p]),
        "orc_decode_weighted_list": (None, [u64p, C.c_uint64, C.c_uint64, C.c_uint, C.c_uint, u32p, u32p]),
        "orc_sssp": (C.c_int, [C.c_uint64, u64p, u32p, u32p, C.c_uint32, i64p]),
        "orc_relabel_row": (None, [u64p, u32p, u32p, u32p, C.c_uint32, u32p]),
        "orc_bfs_labels": (C.c_int, [C.c_uint64, u64p, u32p, C.c_uint32, C.c_int32, _NullableU32,
                                     i32p, i32p]),
        "orc_bfs": (C.c_int, [C.c_uint64, u64p, u32p, C.c_uint32, C.c_int32, i32p, i32p]),
        "orc_bfs_relabeled": (C.c_int, [C.c_uint64, u64p, u32p, C.c_uint32, C.c_int32, i32p, i32p]),
        "orc_pagerank": (C.c_int, [C.c_uint64, u64p, u32p, C.c_double, C.c_uint32, f64p]),
        "orc_pagerank_par": (C.c_int, [C.c_uint64, u64p, u32p, C.c_double, C.c_uint32, f64p, C.c_int]),
        "orc_bfs_levels": (C.c_int, [C.c_uint64, u64p, u32p, C.c_uint32, C.c_int32, _NullableU32, i32p, i32p,
                                     C.c_int]),
        "orc_max_threads": (C.c_int, []),
        "orc_bv_bits": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_bv_plain_build": (None, [u64p, C.c_uint64, C.c_uint64, u64p, u32p, u32p]),
        "orc_bv_plain_get": (C.c_uint64, [u64p, C.c_uint64, C.c_uint64]),
        "orc_bvil_words": (C.c_uint64, [C.c_uint64]),
        "orc_bvil_build": (None, [u64p, C.c_uint64, C.c_uint64, u64p]),
        "orc_bvil_get": (C.c_uint64, [u64p, C.c_uint64, C.c_uint64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _csr(off, col):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    n = off.size - 1
    return n, off, col


# -- widths -------------------------------------------------------------

def bitlen(x: int) -> int:
    return int(lib().orc_bitlen(int(x)))


def global_width(n: int) -> int:
    return int(lib().orc_global_width(int(n)))


def width_field_bits(n: int) -> int:
    return int(lib().orc_width_field_bits(int(n)))


def relabeled_local_widths(off, col, perm, inv):
    """(widths, row lengths) of the relabeled graph, from the original lists."""
    n, off, col = _csr(off, col)
    w = np.zeros(max(n, 1), dtype=np.uint8)
    d = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_relabeled_local_widths(n, off, col, np.ascontiguousarray(perm, np.uint32),
                                     np.ascontiguousarray(inv, np.uint32), w, d)
    return w[:n], d[:n]


def local_widths(off, col) -> np.ndarray:
    n, off, col = _csr(off, col)
    w = np.zeros(n, dtype=np.uint8)
    lib().orc_local_widths(n, off, col, w)
    return w


# -- packing ----------------------------------------------------------

def stream_words(bits: int) -> int:
    return int(lib().orc_stream_words(int(bits)))


def adjacency_bits(off, widths=None, s: int = 0) -> int:
    off = np.ascontiguousarray(off, dtype=np.uint64)
    return int(lib().orc_adjacency_bits(off.size - 1, off, widths, s))


def bit_starts(off, widths=None, s: int = 0) -> np.ndarray:
    off = np.ascontiguousarray(off, dtype=np.uint64)
    P = np.zeros(off.size, dtype=np.uint64)
    lib().orc_bit_starts(off.size - 1, off, widths, s, P)
    return P


def pack_adjacency(off, col, widths=None, s: int = 0) -> np.ndarray:
    n, off, col = _csr(off, col)
    U = adjacency_bits(off, widths, s)
    words = np.zeros(stream_words(U), dtype=np.uint64)
    lib().orc_pack_adjacency(n, off, col, widths, s, words)
    return words


def pack_adjacency_words(off, col, k0: int, k1: int, widths=None, s: int = 0) -> np.ndarray:
    n, off, col = _csr(off, col)
    out = np.zeros(max(k1 - k0, 1), dtype=np.uint64)
    lib().orc_pack_adjacency_words(n, off, col, widths, s, k0, k1, out)
    return out[: k1 - k0]


def gap_widths(off, col) -> np.ndarray:
    """g_v = bl(largest difference of consecutive neighbors) (0 when d_v < 2):
    subsection "Adding Fixed-Size Gap Encoding", local approach."""
    n, off, col = _csr(off, col)
    g = np.zeros(max(n, 1), dtype=np.uint8)
    lib().orc_gap_widths(n, off, col, g)
    return g[:n]


def gap_bit_starts(off, w, g) -> np.ndarray:
    off = np.ascontiguousarray(off, dtype=np.uint64)
    P = np.zeros(off.size, dtype=np.uint64)
    lib().orc_gap_bit_starts(off.size - 1, off, np.ascontiguousarray(w, np.uint8),
                             np.ascontiguousarray(g, np.uint8), P)
    return P


def pack_gap(off, col, w, g) -> np.ndarray:
    n, off, col = _csr(off, col)
    U = int(gap_bit_starts(off, w, g)[-1])
    words = np.zeros(stream_words(U), dtype=np.uint64)
    lib().orc_pack_gap(n, off, col, np.ascontiguousarray(w, np.uint8), np.ascontiguousarray(g, np.uint8), words)
    return words


def decode_gap_list(words, start: int, d: int, w: int, g: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.zeros(max(d, 1), dtype=np.uint32)
    lib().orc_decode_gap_list(words, start, d, w, g, out)
    return out[:d]


def varint_len(x: int) -> int:
    """Bytes of one Varint value (subsection "Incorporating Degree-Minimizing
    (DM)"; base-128, lowest group first)."""
    return int(lib().orc_varint_len(x))


def varint_byte_starts(off, col, diff: bool) -> np.ndarray:
    """Byte start of each Varint list (n + 1 values, the last = stream bytes);
    diff: DMd (first label, then differences), else DMf (every label)."""
    n, off, col = _csr(off, col)
    P = np.zeros(n + 1, dtype=np.uint64)
    lib().orc_varint_byte_starts(n, off, col, int(diff), P)
    return P


def pack_varint(off, col, diff: bool) -> np.ndarray:
    """The Varint byte stream of every list, in vertex order."""
    n, off, col = _csr(off, col)
    total = int(varint_byte_starts(off, col, diff)[-1])
    out = np.zeros(max(total, 1), dtype=np.uint8)
    lib().orc_pack_varint(n, off, col, int(diff), out)
    return out[:total]


def varint_words(stream: np.ndarray) -> np.ndarray:
    """A byte stream as little-endian 64-bit words plus one zero word (byte
    i = bits 8(i mod 8) .. +8 of word floor(i / 8))."""
    nw = (stream.size + 7) // 8 + 1
    buf = np.zeros(nw * 8, dtype=np.uint8)
    buf[: stream.size] = stream
    return buf.view("<u8").astype(np.uint64)


def decode_varint_list(stream, b0: int, b1: int, diff: bool) -> np.ndarray:
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.zeros(max(b1 - b0, 1), dtype=np.uint32)
    cnt = lib().orc_decode_varint_list(stream if stream.size else np.zeros(1, np.uint8), b0, b1, int(diff), out)
    return out[:cnt]


def weight_width(weights) -> int:
    """omega = max(1, bl(largest weight)): one weight width for the graph
    (subsection "Logarithmization of Edge Weights")."""
    wt = np.ascontiguousarray(weights, dtype=np.uint32)
    return int(lib().orc_weight_width(wt.size, wt if wt.size else np.zeros(1, np.uint32)))


def pack_weighted(off, col, weights, widths, s: int, omega: int) -> np.ndarray:
    """Entries of ID then weight (subsection "Accessing an Edge Weight"); the
    ID at w_v bits (widths) or s bits (widths None), the weight at omega."""
    n, off, col = _csr(off, col)
    wt = np.ascontiguousarray(weights, dtype=np.uint32)
    per = (off[1:] - off[:-1]) * ((widths.astype(np.uint64) if widths is not None else np.uint64(s)) + omega)
    U = int(per.sum())
    words = np.zeros(stream_words(U), dtype=np.uint64)
    lib().orc_pack_weighted(n, off, col, wt if wt.size else np.zeros(1, np.uint32),
                            None if widths is None else np.ascontiguousarray(widths, np.uint8), s, omega, words)
    return words


def decode_weighted_list(words, start: int, d: int, w: int, omega: int):
    words = np.ascontiguousarray(words, dtype=np.uint64)
    ids = np.zeros(max(d, 1), dtype=np.uint32)
    wts = np.zeros(max(d, 1), dtype=np.uint32)
    lib().orc_decode_weighted_list(words, start, d, w, omega, ids, wts)
    return ids[:d], wts[:d]


def relabel_weights(off, col, weights, off_new, col_new, perm) -> np.ndarray:
    """The weight of every relabeled entry: new entry (r, c) is the original
    edge (perm[r], perm[c]); the original entries, row by row with ascending
    lists, have ascending keys u * n + x, so a sorted search finds it."""
    n = off.size - 1
    off = np.asarray(off, np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    keys = rows * n + np.asarray(col, np.int64)
    perm = np.asarray(perm, np.int64)
    rows_new = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(off_new, np.int64)))
    want = perm[rows_new] * n + perm[np.asarray(col_new, np.int64)]
    pos = np.searchsorted(keys, want)
    assert np.array_equal(keys[pos], want)
    return np.ascontiguousarray(np.asarray(weights, np.uint32)[pos])


def sssp(off, col, weights, root: int) -> np.ndarray:
    """Shortest-path distances from root (int64, -1 where unreachable), by
    Dijkstra's algorithm: SSSP of section "Considered Algorithms"."""
    n, off, col = _csr(off, col)
    wt = np.ascontiguousarray(weights, dtype=np.uint32)
    dist = np.zeros(max(n, 1), dtype=np.int64)
    rc = lib().orc_sssp(n, off, col, wt if wt.size else np.zeros(1, np.uint32), root, dist)
    if rc != 0:
        raise ValueError(f"orc_sssp failed ({rc})")
    return dist[:n]


def decode_list(words, start: int, d: int, w: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.zeros(max(d, 1), dtype=np.uint32)
    lib().orc_decode_list(words, start, d, w, out)
    return out[:d]


def get_bits(words, start: int, width: int) -> int:
    words = np.ascontiguousarray(words, dtype=np.uint64)
    return int(lib().orc_get_bits(words, start, width))


def pack_fixed(vals, width: int) -> np.ndarray:
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    words = np.zeros(stream_words(vals.size * width), dtype=np.uint64)
    lib().orc_pack_fixed(vals, vals.size, width, words)
    return words


# -- bit vectors ------------------------------------------------------

def rank1(words, i: int) -> int:
    return int(lib().orc_rank1(np.ascontiguousarray(words, dtype=np.uint64), i))


def select1(words, nbits: int, k: int) -> int:
    return int(lib().orc_select1(np.ascontiguousarray(words, dtype=np.uint64), nbits, k))


class EF:
    """Elias-Fano offsets as the oracle builds them."""

    def __init__(self, x, universe: int):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        L = lib()
        self.count = x.size
        self.universe = int(universe)
        self.l = int(L.orc_ef_low_bits(self.count, self.universe))
        self.hbits = int(L.orc_ef_upper_bits(self.count, self.universe, self.l))
        self.low = np.zeros(stream_words(self.count * self.l), dtype=np.uint64)
        self.high = np.zeros(stream_words(self.hbits), dtype=np.uint64)
        self.rank_sb = np.zeros(int(L.orc_ef_rank_entries(self.hbits)), dtype=np.uint32)
        self.sel = np.zeros(max(int(L.orc_ef_select_entries(self.count)), 1), dtype=np.uint32)
        L.orc_ef_build(x, self.count, self.universe, self.low, self.high, self.rank_sb, self.sel)
        self.sel = self.sel[: int(L.orc_ef_select_entries(self.count))]

    def get(self, v: int) -> int:
        return int(lib().orc_ef_get(self.low, self.high, self.hbits, self.l, v))


class PlainBV:
    """bvPL offsets as the oracle builds them: the plain bit vector with the
    one of list v at x_v + v, and its rank/select directory."""

    def __init__(self, x, universe: int):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        L = lib()
        self.count = x.size
        self.universe = int(universe)
        self.nbits = int(L.orc_bv_bits(self.count, self.universe))
        self.bits = np.zeros(stream_words(self.nbits), dtype=np.uint64)
        self.rank_sb = np.zeros(int(L.orc_ef_rank_entries(self.nbits)), dtype=np.uint32)
        self.sel = np.zeros(max(int(L.orc_ef_select_entries(self.count)), 1), dtype=np.uint32)
        L.orc_bv_plain_build(x, self.count, self.universe, self.bits, self.rank_sb, self.sel)
        self.sel = self.sel[: int(L.orc_ef_select_entries(self.count))]

    def get(self, v: int) -> int:
        return int(lib().orc_bv_plain_get(self.bits, self.nbits, v))


class InterleavedBV:
    """bvIL offsets as the oracle builds them: 512-bit blocks of the plain
    bit vector, each preceded by the 64-bit count of ones before it."""

    def __init__(self, x, universe: int):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        L = lib()
        self.count = x.size
        self.universe = int(universe)
        self.nbits = int(L.orc_bv_bits(self.count, self.universe))
        self.words = np.zeros(int(L.orc_bvil_words(self.nbits)), dtype=np.uint64)
        L.orc_bvil_build(x, self.count, self.universe, self.words)

    def get(self, v: int) -> int:
        return int(lib().orc_bvil_get(self.words, self.nbits, v))


# -- relabeling -------------------------------------------------------

def dm_permutation(off):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    n = off.size - 1
    perm = np.zeros(max(n, 1), dtype=np.uint32)
    inv = np.zeros(max(n, 1), dtype=np.uint32)
    lib().orc_dm_permutation(n, off, perm, inv)
    return perm[:n], inv[:n]


def greedy_permutation(off, col):
    """(perm, inv) of the greedy relabeling heuristic (subsection "Adding
    Integer Linear Programming"): vertices by increasing degree hand labels to
    their unlabeled neighbors in list order; edgeless vertices last, by ID."""
    n, off, col = _csr(off, col)
    perm = np.zeros(max(n, 1), dtype=np.uint32)
    inv = np.zeros(max(n, 1), dtype=np.uint32)
    lib().orc_greedy_permutation(n, off, col, perm, inv)
    return perm[:n], inv[:n]


def relabel(off, col, perm, inv):
    n, off, col = _csr(off, col)
    off2 = np.zeros(n + 1, dtype=np.uint64)
    col2 = np.zeros(max(col.size, 1), dtype=np.uint32)
    lib().orc_relabel(n, off, col, np.ascontiguousarray(perm, np.uint32),
                      np.ascontiguousarray(inv, np.uint32), off2, col2)
    return off2, col2[: col.size]


def relabel_row(off, col, perm, inv, x: int) -> np.ndarray:
    n, off, col = _csr(off, col)
    v = int(perm[x])
    d = int(off[v + 1] - off[v])
    out = np.zeros(max(d, 1), dtype=np.uint32)
    lib().orc_relabel_row(off, col, np.ascontiguousarray(perm, np.uint32),
                          np.ascontiguousarray(inv, np.uint32), x, out)
    return out[:d]


# -- algorithms -------------------------------------------------------

def bfs(off, col, root: int, max_depth: int = -1, relabeled: bool = False, labels=None):
    n, off, col = _csr(off, col)
    depth = np.zeros(max(n, 1), dtype=np.int32)
    parent = np.zeros(max(n, 1), dtype=np.int32)
    if relabeled:
        rc = lib().orc_bfs_relabeled(n, off, col, root, max_depth, depth, parent)
    elif labels is not None:
        rc = lib().orc_bfs_labels(n, off, col, root, max_depth,
                                  np.ascontiguousarray(labels, np.uint32), depth, parent)
    else:
        rc = lib().orc_bfs(n, off, col, root, max_depth, depth, parent)
    if rc != 0:
        raise ValueError(f"oracle bfs failed ({rc})")
    return depth[:n], parent[:n]


def pagerank(off, col, alpha: float = 0.85, iters: int = 20) -> np.ndarray:
    n, off, col = _csr(off, col)
    pr = np.zeros(max(n, 1), dtype=np.float64)
    rc = lib().orc_pagerank(n, off, col, alpha, iters, pr)
    if rc != 0:
        raise ValueError("oracle pagerank failed")
    return pr[:n]


def pagerank_par(off, col, alpha: float = 0.85, iters: int = 20, threads: int = 0) -> np.ndarray:
    """pagerank() on every host core (threads <= 0: OpenMP's default);
    bit-identical to the one-thread result."""
    n, off, col = _csr(off, col)
    pr = np.zeros(max(n, 1), dtype=np.float64)
    rc = lib().orc_pagerank_par(n, off, col, alpha, iters, pr, int(threads))
    if rc != 0:
        raise ValueError("oracle pagerank_par failed")
    return pr[:n]


def bfs_levels(off, col, root: int, max_depth: int = -1, labels=None, threads: int = 0):
    """Level-synchronous BFS on every host core: the same depths and parents
    as bfs() (labels: the stored label of every vertex for the parent rule,
    e.g. the inverse degree permutation; None: the IDs themselves)."""
    n, off, col = _csr(off, col)
    depth = np.zeros(max(n, 1), dtype=np.int32)
    parent = np.zeros(max(n, 1), dtype=np.int32)
    lab = None if labels is None else np.ascontiguousarray(labels, np.uint32)
    rc = lib().orc_bfs_levels(n, off, col, root, max_depth, lab, depth, parent, int(threads))
    if rc != 0:
        raise ValueError(f"oracle bfs_levels failed ({rc})")
    return depth[:n], parent[:n]


def max_threads() -> int:
    """Threads the all-core oracle functions use by default."""
    return int(lib().orc_max_threads())


# -- the whole encoding as the oracle defines it --------------------

class Encoding:
    """Every array of the packed representation, built by the oracle.

    id_mode: "global" (every ID at s bits), "local" (list v at w_v bits,
    with a width table at F bits per vertex), "local-gap" (first element at
    w_v bits, the differences at g_v bits, both tables at F bits),
    "varint-full" or "varint-diff" (a byte stream of Varint labels or of a
    first label and differences; offsets are byte starts).  offset_mode: "packed"
    (fixed-width offsets), "ef" (Elias-Fano with rank/select directory),
    "plain-bv" (bvPL: plain bit vector with a rank/select directory) or
    "interleaved-bv" (bvIL: the bit vector with interleaved 64-bit counts).
    The offset values are element offsets O[v] in global mode (bit start =
    s * O[v]) and bit starts P_v in local mode.  relabel: False, True or
    "degree" (the degree-minimizing permutation), or "greedy" (the greedy
    heuristic), applied first."""

    def __init__(self, off, col, id_mode="global", offset_mode="packed", relabel=False, weights=None):
        n, off, col = _csr(off, col)
        self.n = n
        self.m = col.size
        self.omega = 0
        self.weights = None
        if weights is not None:
            if id_mode not in ("global", "local"):
                raise ValueError("weighted encodings: global or local IDs")
            self.weights = np.ascontiguousarray(weights, dtype=np.uint32)
            self.omega = weight_width(self.weights)
        if relabel:
            if relabel == "greedy":
                self.perm, self.inv = greedy_permutation(off, col)
            else:
                self.perm, self.inv = dm_permutation(off)
            off0, col0 = off, col
            off, col = globals()["relabel"](off, col, self.perm, self.inv)
            if self.weights is not None:
                self.weights = relabel_weights(off0, col0, self.weights, off, col, self.perm)
        else:
            self.perm = self.inv = None
        self.off, self.col = off, col
        self.s = global_width(n)
        self.gwidths = None
        self.stream = None
        if id_mode in ("varint-full", "varint-diff"):
            self.diff = id_mode == "varint-diff"
            self.widths = None
            self.stream = pack_varint(off, col, self.diff)
            self.A = varint_words(self.stream)
            self.U = 8 * self.stream.size
            vals = varint_byte_starts(off, col, self.diff)
            universe = self.stream.size
        elif id_mode == "global":
            self.widths = None
            self.U = adjacency_bits(off, None, self.s + self.omega)
            if self.weights is None:
                self.A = pack_adjacency(off, col, None, self.s)
            else:
                self.A = pack_weighted(off, col, self.weights, None, self.s, self.omega)
            vals = off
            universe = self.m
        elif id_mode == "local-gap":
            self.widths = local_widths(off, col)
            self.gwidths = gap_widths(off, col)
            self.F = width_field_bits(n)
            self.W = pack_fixed(self.widths.astype(np.uint64), self.F)
            self.G = pack_fixed(self.gwidths.astype(np.uint64), self.F)
            P = gap_bit_starts(off, self.widths, self.gwidths)
            self.U = int(P[-1])
            self.A = pack_gap(off, col, self.widths, self.gwidths)
            vals = P
            universe = self.U
        else:
            self.widths = local_widths(off, col)
            self.F = width_field_bits(n)
            self.W = pack_fixed(self.widths.astype(np.uint64), self.F)
            if self.weights is None:
                ew = self.widths
                self.A = pack_adjacency(off, col, self.widths, 0)
            else:  # an entry takes w_v + omega bits (0 for an empty list)
                ew = np.where(off[1:] > off[:-1], self.widths.astype(np.int64) + self.omega, 0).astype(np.uint8)
                self.A = pack_weighted(off, col, self.weights, self.widths, 0, self.omega)
            self.U = adjacency_bits(off, ew, 0)
            vals = bit_starts(off, ew, 0)
            universe = self.U
        if self.stream is not None:
            self.P = vals
        elif self.gwidths is None and self.widths is None:
            self.P = bit_starts(off, None, self.s + self.omega)
        elif self.gwidths is None:
            self.P = vals
        else:
            self.P = vals
        self.offset_values = vals
        self.universe = universe
        self.ef = self.bv = self.bvil = None
        if offset_mode == "packed":
            self.wO = bitlen(universe)
            self.O = pack_fixed(vals, self.wO)
        elif offset_mode == "plain-bv":
            self.bv = PlainBV(vals, universe)
        elif offset_mode == "interleaved-bv":
            self.bvil = InterleavedBV(vals, universe)
        else:
            self.ef = EF(vals, universe)

    def weights_of(self, x: int) -> np.ndarray:
        """Weights of the stored list of x, decoded bit by bit."""
        w = self.s if self.widths is None else int(self.widths[x])
        d = int(self.off[x + 1] - self.off[x])
        return decode_weighted_list(self.A, int(self.P[x]), d, w, self.omega)[1]

    def neighbors(self, x: int) -> np.ndarray:
        """Stored list of stored label x, decoded bit by bit."""
        if self.stream is not None:
            return decode_varint_list(self.stream, int(self.P[x]), int(self.P[x + 1]), self.diff)
        w = self.s if self.widths is None else int(self.widths[x])
        d = int(self.off[x + 1] - self.off[x])
        if self.weights is not None:
            return decode_weighted_list(self.A, int(self.P[x]), d, w, self.omega)[0]
        if self.gwidths is not None:
            return decode_gap_list(self.A, int(self.P[x]), d, w, int(self.gwidths[x]))
        return decode_list(self.A, int(self.P[x]), d, w)
