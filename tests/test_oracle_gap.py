"""Pins of the oracle's fixed-size gap encoding (subsection "Adding
Fixed-Size Gap Encoding", local approach): per list the first element at the
local width w_v = max(1, bl(max N_v)) and every difference of consecutive
neighbors at g_v = bl(largest difference) bits."""

import numpy as np
import pytest

import oracle as orc
from paper_2010_15879_amd import graphgen as gg


def test_gap_hand_example():
    # one list [3, 5, 6, 10] (vertex 0 of a star-like graph): w = bl(10) = 4,
    # differences 2, 1, 4 -> g = bl(4) = 3; 4 + 3*3 = 13 bits:
    # 3 | 2 << 4 | 1 << 7 | 4 << 10 = 4259
    edges = [(0, 3), (0, 5), (0, 6), (0, 10)]
    off, col = gg.csr_from_edges(11, edges).numpy()
    e = orc.Encoding(off, col, "local-gap", "packed")
    assert int(e.widths[0]) == 4 and int(e.gwidths[0]) == 3
    assert int(e.P[1] - e.P[0]) == 13
    assert int(e.A[0]) & ((1 << 13) - 1) == 4259
    # every other list has one element (the hub 0): first element only, g = 0
    for v in (3, 5, 6, 10):
        assert int(e.gwidths[v]) == 0 and int(e.P[v + 1] - e.P[v]) == 1  # bl(0) -> width 1
    np.testing.assert_array_equal(e.neighbors(0), [3, 5, 6, 10])


def bigint_gap_stream(off, col):
    """The stream as one Python integer: first element, then differences."""
    x, pos = 0, 0
    n = off.size - 1
    for v in range(n):
        a = [int(c) for c in col[off[v]:off[v + 1]]]
        if not a:
            continue
        w = max(1, max(a).bit_length())
        g = max((a[i] - a[i - 1] for i in range(1, len(a))), default=0).bit_length()
        x |= a[0] << pos
        pos += w
        for i in range(1, len(a)):
            x |= (a[i] - a[i - 1]) << pos
            pos += g
    return x, pos


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gap_stream_matches_bigint(seed):
    g = gg.kronecker(8, 8, seed=seed)
    off, col = g.numpy()
    e = orc.Encoding(off, col, "local-gap", "packed")
    x, bits = bigint_gap_stream(off.astype(np.int64), col)
    assert e.U == bits
    got = 0
    for i, wd in enumerate(e.A):
        got |= int(wd) << (64 * i)
    assert got == x
    assert int(e.A[-1]) == 0  # the zero pad word


def test_gap_bits_closed_form():
    # a path keeps every difference at 1 (g = 1) except for end vertices
    n = 300
    off, col = gg.csr_from_edges(n, [(i, i + 1) for i in range(n - 1)]).numpy()
    e = orc.Encoding(off, col, "local-gap", "ef")
    # inner vertex v: list [v-1, v+1]: w = bl(v+1), one difference of 2 -> g = 2
    for v in (1, 7, 200):
        assert int(e.gwidths[v]) == 2
        assert int(e.P[v + 1] - e.P[v]) == (v + 1).bit_length() + 2


@pytest.mark.parametrize("seed", [4, 5])
def test_gap_roundtrip(seed):
    g = gg.erdos_renyi(9, 6, seed=seed)
    off, col = g.numpy()
    for om in ("packed", "ef"):
        e = orc.Encoding(off, col, "local-gap", om)
        for v in range(0, g.n, 7):
            np.testing.assert_array_equal(e.neighbors(v), col[off[v]:off[v + 1]])
