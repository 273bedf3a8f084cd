"""Pins of the oracle's Varint lists (subsection "Incorporating
Degree-Minimizing (DM)": DMf stores full labels, DMd a first label and then
differences, each as a Varint).  Byte layout read as the common base-128
form: 7 value bits per byte, lowest group first, the top bit set on every
byte of a value but its last."""

import numpy as np
import pytest

import oracle as orc
from paper_2010_15879_amd import graphgen as gg


def stream_of(n, edges, diff):
    off, col = gg.csr_from_edges(n, edges).numpy()
    return orc.pack_varint(off, col, diff), off, col


@pytest.mark.parametrize("x,expect", [
    (0, [0x00]), (1, [0x01]), (127, [0x7F]), (128, [0x80, 0x01]), (300, [0xAC, 0x02]),
    (16383, [0xFF, 0x7F]), (16384, [0x80, 0x80, 0x01]), (2**31 - 1, [0xFF, 0xFF, 0xFF, 0xFF, 0x07]),
])
def test_single_values(x, expect):
    # vertex 0's only neighbor is x (x > 0), or vertex 1's only neighbor is 0
    if x == 0:
        s, _, _ = stream_of(2, [(0, 1)], diff=False)
        assert list(s) == [0x01, 0x00]
        return
    if x >= 1 << 20:
        # too many vertices for a graph: the value itself through the length
        # function and a two-vertex list built around it is enough
        assert orc.varint_len(x) == len(expect)
        assert closed_form_bytes(x) == expect
        stream = np.array(expect, np.uint8)
        np.testing.assert_array_equal(orc.decode_varint_list(stream, 0, stream.size, False), [x])
        return
    s, _, _ = stream_of(x + 1, [(0, x)], diff=False)
    # list 0 = [x]; list x = [0]; every other list is empty
    assert list(s) == expect + [0x00]
    assert orc.varint_len(x) == len(expect)


def test_hand_lists():
    # vertex 0 with neighbors 3, 5, 6, 10; each of those with neighbor 0
    edges = [(0, 3), (0, 5), (0, 6), (0, 10)]
    s, off, col = stream_of(11, edges, diff=True)
    assert list(s) == [3, 2, 1, 4, 0, 0, 0, 0]
    s, _, _ = stream_of(11, edges, diff=False)
    assert list(s) == [3, 5, 6, 10, 0, 0, 0, 0]
    # a difference of two bytes: [1, 200] -> DMd 1, 199; DMf 1, 200
    s, _, _ = stream_of(201, [(0, 1), (0, 200)], diff=True)
    assert list(s[:3]) == [0x01, 0xC7, 0x01]
    s, _, _ = stream_of(201, [(0, 1), (0, 200)], diff=False)
    assert list(s[:3]) == [0x01, 0xC8, 0x01]


def test_words_little_endian():
    s, _, _ = stream_of(301, [(0, 300)], diff=False)
    w = orc.varint_words(s)
    assert w.size == 2 and int(w[0]) == 0x02AC and int(w[1]) == 0


def test_byte_starts_and_encoding_arrays():
    edges = [(0, 3), (0, 5), (0, 6), (0, 10)]
    off, col = gg.csr_from_edges(11, edges).numpy()
    e = orc.Encoding(off, col, "varint-diff", "packed")
    np.testing.assert_array_equal(e.P, [0, 4, 4, 4, 5, 5, 6, 7, 7, 7, 7, 8])
    assert e.U == 64 and e.universe == 8
    np.testing.assert_array_equal(e.neighbors(0), [3, 5, 6, 10])


def closed_form_bytes(x: int) -> list:
    """Varint bytes of x written from the definition: L = max(1, ceil(bl(x)/7))
    groups, group k = bits 7k..7k+6, top bit on all groups but the last."""
    L = max(1, -(-x.bit_length() // 7))
    return [((x >> (7 * k)) & 127) | (128 if k < L - 1 else 0) for k in range(L)]


@pytest.mark.parametrize("diff", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_stream_closed_form(seed, diff):
    """The whole stream equals the concatenation of the closed-form bytes."""
    g = gg.kronecker(10, 8, seed=seed)
    off, col = g.numpy()
    s = orc.pack_varint(off, col, diff)
    expect = []
    for v in range(g.n):
        row = [int(x) for x in col[off[v]:off[v + 1]]]
        for i, x in enumerate(row):
            expect += closed_form_bytes(x - row[i - 1] if diff and i else x)
    np.testing.assert_array_equal(s, np.array(expect, np.uint8))
    P = orc.varint_byte_starts(off, col, diff)
    # a value ends at each byte with the top bit clear: one per entry
    for v in range(0, g.n, 37):
        seg = s[P[v]:P[v + 1]]
        assert int((seg < 128).sum()) == off[v + 1] - off[v]


@pytest.mark.parametrize("diff", [False, True])
def test_round_trip(diff):
    g = gg.erdos_renyi(11, 12, seed=4)
    off, col = g.numpy()
    e = orc.Encoding(off, col, "varint-diff" if diff else "varint-full", "ef")
    for v in range(g.n):
        np.testing.assert_array_equal(e.neighbors(v), col[off[v]:off[v + 1]])


def test_dmd_not_larger_than_dmf():
    g = gg.kronecker(11, 16, seed=5)
    off, col = g.numpy()
    for rl in (False, True):
        f = orc.Encoding(off, col, "varint-full", "packed", rl)
        d = orc.Encoding(off, col, "varint-diff", "packed", rl)
        assert d.U <= f.U
    # the degree relabeling gives hubs the shortest labels: DMf shrinks
    assert orc.Encoding(off, col, "varint-full", "packed", True).U <= orc.Encoding(off, col, "varint-full",
                                                                                 "packed", False).U


def test_large_values_two_vertex_list():
    """A value of 4 and 5 bytes inside a list, through the list decoder."""
    big = [(1 << 21) + 5, (1 << 28) + 3]
    stream = np.array(sum((closed_form_bytes(x) for x in [7, big[0] - 7, big[1] - big[0]]), []), np.uint8)
    np.testing.assert_array_equal(orc.decode_varint_list(stream, 0, stream.size, True), [7] + big)
    stream = np.array(sum((closed_form_bytes(x) for x in [7] + big), []), np.uint8)
    np.testing.assert_array_equal(orc.decode_varint_list(stream, 0, stream.size, False), [7] + big)
    assert orc.varint_len(big[0]) == 4 and orc.varint_len(big[1]) == 5
