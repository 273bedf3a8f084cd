"""Seeded synthetic graph inputs (Kronecker/R-MAT and Erdos-Renyi).

This module only manufactures inputs: edge lists, their canonical
undirected CSR form and BFS roots.  It contains none of the representation's
arithmetic (no widths, packing, offsets, traversal or ranking), so the CPU
oracle and the GPU library can both be fed from it without sharing code.

The evaluation section of the paper (subsection "Considered Graphs") uses
Kronecker graphs named sX_eY (X = log2 n, Y = average edges per vertex) and
Erdos-Renyi uniform graphs; the datasets themselves are not available, so the
generators below stand in for them.

Randomness comes from one counter-based generator, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): value i
of stream `key` is mix64(key + (i + 1) * 0x9E3779B97F4A7C15).  Every draw is a
pure function of (seed, stream, index), so the same graph comes out on the CPU
and on a GPU, in any chunking.  All arithmetic is done in torch int64 with
explicit masking for the logical shifts.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

_MASK64 = (1 << 64) - 1


def _s64(x: int) -> int:
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_MIX1 = _s64(0xBF58476D1CE4E5B9)
_MIX2 = _s64(0x94D049BB133111EB)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 lanes viewed as uint64."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on int64 lanes (wrap-around arithmetic)."""
    z = (z ^ _srl(z, 30)) * _MIX1
    z = (z ^ _srl(z, 27)) * _MIX2
    return z ^ _srl(z, 31)


def mix64_int(z: int) -> int:
    """Same output function on Python integers (used to derive stream keys)."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """Key of an independent SplitMix64 stream derived from (seed, stream)."""
    return mix64_int(mix64_int(seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) ^ (stream * 0xD1B54A32D192ED03))


def splitmix_at(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Value number idx (0-based) of the SplitMix64 sequence started at key."""
    return mix64(idx * _GOLDEN + _s64(key + 0x9E3779B97F4A7C15))


def uniform53(key: int, idx: torch.Tensor) -> torch.Tensor:
    """53-bit uniform integers in [0, 2^53) from the stream."""
    return _srl(splitmix_at(key, idx), 11)


# ---------------------------------------------------------------------------
# edge generators
# ---------------------------------------------------------------------------

RMAT_ABC = (0.57, 0.19, 0.19)

_STREAM_RMAT = 1
_STREAM_SCRAMBLE = 2
_STREAM_ER = 3
_STREAM_ROOTS = 4
_STREAM_WEIGHTS = 6


def _scramble(v: torch.Tensor, scale: int, seed: int) -> torch.Tensor:
    """Seeded bijection of [0, 2^scale): two rounds of odd multiply + add and
    an xor-shift, each invertible modulo 2^scale."""
    if scale == 0:
        return v
    mask = (1 << scale) - 1
    k = stream_key(seed, _STREAM_SCRAMBLE)
    for r in range(2):
        mul = (mix64_int(k + 2 * r) | 1) & mask
        add = mix64_int(k + 2 * r + 1) & mask
        v = (v * mul + add) & mask
        v = v ^ (v >> ((scale + 1) // 2))
    return v


def rmat_edges(scale: int, edge_factor: int, seed: int, device="cpu",
               chunk: int = 1 << 24, abc=RMAT_ABC, scramble: bool = True):
    """R-MAT edge list with edge_factor * 2^scale directed samples.

    For every edge and every one of `scale` levels one quadrant is chosen with
    probabilities (a, b, c, d); the source takes the row bit and the target the
    column bit.  No noise is added.  IDs are then scrambled by a seeded
    bijection so that degree does not follow the label."""
    n = 1 << scale
    e_total = edge_factor * n
    a, b, c = abc
    one = 1 << 53
    ta = int(a * one)
    tab = int((a + b) * one)
    tabc = int((a + b + c) * one)
    key = stream_key(seed, _STREAM_RMAT)
    srcs, dsts = [], []
    for e0 in range(0, e_total, chunk):
        e1 = min(e_total, e0 + chunk)
        e = torch.arange(e0, e1, dtype=torch.int64, device=device)
        src = torch.zeros_like(e)
        dst = torch.zeros_like(e)
        for lvl in range(scale):
            r = uniform53(key, e * scale + lvl)
            row = (r >= tab).to(torch.int64)            # quadrants c, d
            col = ((r >= ta) & (r < tab)) | (r >= tabc)  # quadrants b, d
            bit = scale - 1 - lvl
            src |= row << bit
            dst |= col.to(torch.int64) << bit
        srcs.append(src)
        dsts.append(dst)
    src = torch.cat(srcs) if srcs else torch.zeros(0, dtype=torch.int64, device=device)
    dst = torch.cat(dsts) if dsts else torch.zeros(0, dtype=torch.int64, device=device)
    if scramble:
        src = _scramble(src, scale, seed)
        dst = _scramble(dst, scale, seed)
    return n, src, dst


def er_edges(scale: int, edge_factor: int, seed: int, device="cpu", chunk: int = 1 << 24):
    """Uniform random edge list: edge_factor * 2^scale pairs on [0, n)^2."""
    n = 1 << scale
    e_total = edge_factor * n
    key = stream_key(seed, _STREAM_ER)
    mask = n - 1
    srcs, dsts = [], []
    for e0 in range(0, e_total, chunk):
        e1 = min(e_total, e0 + chunk)
        e = torch.arange(e0, e1, dtype=torch.int64, device=device)
        srcs.append(_srl(splitmix_at(key, 2 * e), 11) & mask)
        dsts.append(_srl(splitmix_at(key, 2 * e + 1), 11) & mask)
    src = torch.cat(srcs) if srcs else torch.zeros(0, dtype=torch.int64, device=device)
    dst = torch.cat(dsts) if dsts else torch.zeros(0, dtype=torch.int64, device=device)
    return n, src, dst


# ---------------------------------------------------------------------------
# canonical undirected CSR
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CSR:
    """Canonical undirected graph: both directions stored, no self-loops, no
    duplicates, every neighbor list strictly increasing.  row_offsets is
    int64[n+1], col is int32[M] (IDs < 2^31)."""
    n: int
    row_offsets: torch.Tensor
    col: torch.Tensor

    @property
    def m(self) -> int:
        return int(self.col.numel())

    def degrees(self) -> torch.Tensor:
        return self.row_offsets[1:] - self.row_offsets[:-1]

    def to(self, device) -> "CSR":
        return CSR(self.n, self.row_offsets.to(device), self.col.to(device))

    def numpy(self):
        return self.row_offsets.cpu().numpy(), self.col.cpu().numpy()


def canonical_csr(n: int, src: torch.Tensor, dst: torch.Tensor) -> CSR:
    """Edge list -> both directions -> drop self-loops -> drop duplicates ->
    sort by (src, dst) -> CSR."""
    if n >= (1 << 31):
        raise ValueError("vertex IDs must fit in 31 bits")
    keep = src != dst
    s = src[keep]
    d = dst[keep]
    key = torch.cat([s * n + d, d * n + s])
    del s, d, keep
    # sort in source ranges of at most 2^30 keys each (large graphs), so that no
    # single sort exceeds 32-bit indexing; the concatenation is globally sorted
    parts = max(1, -(-key.numel() // (1 << 30)))
    if parts == 1:
        key = torch.unique(key, sorted=True)
    else:
        bounds = [(n * i) // parts for i in range(parts + 1)]
        chunks = []
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            sel = key[(key >= lo * n) & (key < hi * n)]
            chunks.append(torch.unique(sel, sorted=True))
            del sel
        del key
        key = torch.cat(chunks)
        del chunks
    # row v starts at the first key >= v * n
    offs = torch.searchsorted(key, torch.arange(n + 1, dtype=torch.int64, device=key.device) * n)
    col = torch.remainder(key, n).to(torch.int32)
    del key
    return CSR(n, offs.to(torch.int64), col)


def csr_from_edges(n: int, edges, device="cpu") -> CSR:
    """Canonical CSR from a small Python list of (u, v) pairs."""
    if len(edges) == 0:
        z = torch.zeros(0, dtype=torch.int64, device=device)
        return canonical_csr(n, z, z)
    e = torch.tensor(edges, dtype=torch.int64, device=device).reshape(-1, 2)
    return canonical_csr(n, e[:, 0].contiguous(), e[:, 1].contiguous())


def kronecker(scale: int, edge_factor: int = 16, seed: int = 1, device="cpu") -> CSR:
    n, s, d = rmat_edges(scale, edge_factor, seed, device=device)
    return canonical_csr(n, s, d)


def erdos_renyi(scale: int, edge_factor: int = 16, seed: int = 1, device="cpu") -> CSR:
    n, s, d = er_edges(scale, edge_factor, seed, device=device)
    return canonical_csr(n, s, d)


def edge_weights(g: CSR, max_weight: int = 255, seed: int = 1) -> torch.Tensor:
    """int32 weight in [1, max_weight] for every stored entry of g, the same
    for both directions of an edge (drawn from the stream at the index of the
    unordered pair): uniform integer weights as the GAP suite draws them for
    weighted Kronecker graphs."""
    dev = g.col.device
    deg = g.row_offsets[1:] - g.row_offsets[:-1]
    src = torch.repeat_interleave(torch.arange(g.n, device=dev, dtype=torch.int64), deg)
    dst = g.col.to(torch.int64)
    pair = torch.minimum(src, dst) * g.n + torch.maximum(src, dst)
    del src, dst
    r = uniform53(stream_key(seed, _STREAM_WEIGHTS), pair)
    return (1 + r % max_weight).to(torch.int32)


def pick_roots(g: CSR, count: int = 64, seed: int = 1) -> list:
    """`count` distinct non-isolated vertices, uniformly at random: the
    vertices with the smallest SplitMix64 draws, in draw order."""
    deg = g.degrees()
    cand = torch.nonzero(deg > 0).flatten()
    if cand.numel() == 0:
        return []
    key = stream_key(seed, _STREAM_ROOTS)
    h = _srl(splitmix_at(key, cand), 1)  # non-negative 63-bit keys
    order = torch.argsort(h)[: min(count, cand.numel())]
    return [int(x) for x in cand[order].cpu().tolist()]


def random_graph(n: int, p: float, seed: int, device="cpu") -> CSR:
    """Small G(n, p) graph for tests: each unordered pair kept with prob p."""
    if n <= 1:
        return csr_from_edges(max(n, 1), [], device)
    iu = torch.triu_indices(n, n, offset=1, device=device)
    key = stream_key(seed, 5)
    r = uniform53(key, torch.arange(iu.shape[1], dtype=torch.int64, device=device))
    keep = r < int(p * (1 << 53))
    return canonical_csr(n, iu[0][keep].contiguous(), iu[1][keep].contiguous())
