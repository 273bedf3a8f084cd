"""Pins of the oracle's plain (bvPL) and interleaved (bvIL) bit-vector
offsets (subsection "Arrays of Offsets vs. Bit Vectors for O" and the table
of offset structures): hand-worked words (tests/golden/bv_small.txt), the
closed-form sizes of the table (u + n + 1 bits; bvIL adds one 64-bit count
per 512 bits), numpy brute force for the positions of the ones, rank and
select, the special case where the Elias-Fano upper bits are the same
vector (no low bits), and every offset recovered from both layouts."""

import numpy as np
import pytest

import oracle as orc
from paper_2010_15879_amd import graphgen as gg


def bits_of(words, nbits):
    """Bit b of a stream = bit (b mod 64) of word b // 64."""
    w = np.asarray(words, dtype=np.uint64)
    b = np.arange(nbits, dtype=np.uint64)
    return ((w[(b >> np.uint64(6)).astype(np.int64)] >> (b & np.uint64(63))) & np.uint64(1)).astype(np.int64)


@pytest.mark.parametrize("k", ["1", "2"])
def test_golden(golden, k):
    fx = golden("bv_small.txt")
    x = np.array(fx["x" + k], dtype=np.uint64)
    u = fx["u" + k][0]
    pl = orc.PlainBV(x, u)
    assert pl.nbits == fx["bits" + k][0]
    if "plain_words" + k in fx:
        assert pl.bits.tolist() == fx["plain_words" + k]
    else:
        nz = fx["plain_nonzero" + k]
        want = np.zeros(pl.bits.size, dtype=np.uint64)
        for i in range(0, len(nz), 2):
            want[nz[i]] = nz[i + 1]
        assert pl.bits.tolist() == want.tolist()
    assert pl.rank_sb.tolist() == fx["rank" + k]
    assert pl.sel.tolist() == fx["sel" + k]
    il = orc.InterleavedBV(x, u)
    assert il.words.tolist() == fx["il_words" + k]
    for v in range(x.size):
        assert pl.get(v) == int(x[v]) == il.get(v)


def random_offsets(n, max_len, seed, empty=0.3):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, size=n)
    lens[rng.random(n) < empty] = 0
    x = np.zeros(n + 1, dtype=np.uint64)
    x[1:] = np.cumsum(lens)
    return x


@pytest.mark.parametrize("seed,n,max_len", [(1, 1, 0), (2, 7, 3), (3, 200, 40), (4, 1000, 3), (5, 3000, 700),
                                            (6, 64, 0), (7, 65, 1), (8, 4096, 17)])
def test_brute_force(seed, n, max_len):
    x = random_offsets(n, max_len, seed)
    u = int(x[-1])
    pl = orc.PlainBV(x, u)
    # closed forms of the table: u + n + 1 bits, n + 1 ones
    assert pl.nbits == u + x.size
    b = bits_of(pl.bits, pl.nbits)
    assert int(b.sum()) == x.size
    ones = np.flatnonzero(b)
    np.testing.assert_array_equal(ones - np.arange(x.size), x.astype(np.int64))  # select1(v) - v = x_v
    # words past the last bit (the pad word included) are zero
    assert not np.any(bits_of(pl.bits, pl.bits.size * 64)[pl.nbits:])
    # directory: rank1(512 b) and select1(64 j), by numpy
    cum = np.concatenate([[0], np.cumsum(b)])
    nr = (pl.nbits + 511) // 512 + 1
    want_rank = [int(cum[min(512 * i, pl.nbits)]) for i in range(nr - 1)] + [x.size]
    assert pl.rank_sb.tolist() == want_rank
    assert pl.sel.tolist() == ones[::64].tolist()
    # bvIL: count words = ones before each block, data words = the vector
    il = orc.InterleavedBV(x, u)
    blocks = (pl.nbits + 511) // 512
    assert il.words.size == 9 * blocks + 1
    for j in range(blocks):
        assert int(il.words[9 * j]) == int(cum[512 * j])
        data = pl.bits[8 * j: 8 * j + 8]
        np.testing.assert_array_equal(il.words[9 * j + 1: 9 * j + 1 + data.size], data)
        assert not np.any(il.words[9 * j + 1 + data.size: 9 * j + 9])
    assert int(il.words[-1]) == x.size
    for v in range(0, x.size, max(1, x.size // 50)):
        assert pl.get(v) == int(x[v]) == il.get(v)


def test_no_low_bits_equals_elias_fano_upper_bits():
    # when the universe is below the number of values, Elias-Fano keeps no
    # low bits and its upper bit vector is this plain vector
    x = random_offsets(500, 1, seed=9, empty=0.6)
    assert int(x[-1]) < x.size
    ef = orc.EF(x, int(x[-1]))
    pl = orc.PlainBV(x, int(x[-1]))
    assert ef.l == 0 and ef.hbits == pl.nbits
    np.testing.assert_array_equal(ef.high, pl.bits)
    np.testing.assert_array_equal(ef.rank_sb, pl.rank_sb)
    np.testing.assert_array_equal(ef.sel, pl.sel)


@pytest.mark.parametrize("ids", ["global", "local"])
def test_encodings_of_a_graph(ids):
    g = gg.kronecker(10, 8, seed=2)
    off, col = g.numpy()
    for mode in ("plain-bv", "interleaved-bv"):
        e = orc.Encoding(off, col, id_mode=ids, offset_mode=mode)
        st = e.bv if mode == "plain-bv" else e.bvil
        assert st.nbits == e.universe + g.n + 1
        for v in range(0, g.n + 1, 37):
            assert st.get(v) == int(e.offset_values[v])
    # sizes of the table for this graph: bvIL = bvPL's vector + 64 bits per 512
    pl = orc.Encoding(off, col, id_mode=ids, offset_mode="plain-bv").bv
    il = orc.Encoding(off, col, id_mode=ids, offset_mode="interleaved-bv").bvil
    assert il.words.size * 64 == 9 * 64 * ((pl.nbits + 511) // 512) + 64
