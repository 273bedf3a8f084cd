"""Seeded synthetic inputs: the counter-based generator matches its
published definition, and the canonical CSR has the stated structure."""

import numpy as np
import torch

from paper_2010_15879_amd import graphgen as gg

M64 = (1 << 64) - 1


def splitmix64_reference(seed, count):
    """SplitMix64 as published: state += 0x9E3779B97F4A7C15, then mix."""
    out, state = [], seed & M64
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def test_splitmix_matches_published_definition():
    for key in [0, 1, 1234567, (1 << 63) + 17, M64]:
        got = gg.splitmix_at(key, torch.arange(50, dtype=torch.int64))
        want = splitmix64_reference(key, 50)
        assert [int(x) & M64 for x in got.tolist()] == want


def test_kronecker_canonical_structure():
    g = gg.kronecker(12, 16, seed=1)
    off, col = g.numpy()
    n, m = g.n, g.m
    assert off[0] == 0 and off[-1] == m and m % 2 == 0
    src = np.repeat(np.arange(n), np.diff(off))
    k = src.astype(np.int64) * n + col
    assert np.all(np.diff(k) > 0)                      # sorted, no duplicates
    assert not np.any(src == col)                      # no self-loops
    kt = col.astype(np.int64) * n + src
    assert np.array_equal(np.sort(kt), k)              # symmetric
    deg = np.diff(off)
    assert deg.max() > 20 * deg.mean()                 # power-law hubs
    assert 0.15 < (deg == 0).mean() < 0.4              # isolated share of R-MAT


def test_generators_are_deterministic_and_chunk_free():
    a = gg.rmat_edges(10, 4, seed=3, chunk=1 << 20)
    b = gg.rmat_edges(10, 4, seed=3, chunk=777)
    assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    c = gg.er_edges(10, 4, seed=3, chunk=1000)
    d = gg.er_edges(10, 4, seed=3)
    assert torch.equal(c[1], d[1]) and torch.equal(c[2], d[2])


def test_scramble_is_bijective():
    for scale in [1, 5, 12]:
        v = torch.arange(1 << scale, dtype=torch.int64)
        s = gg._scramble(v, scale, seed=9)
        assert torch.equal(torch.sort(s).values, v)


def test_roots_distinct_non_isolated():
    g = gg.kronecker(12, 16, seed=1)
    roots = gg.pick_roots(g, 64, seed=1)
    deg = g.degrees()
    assert len(set(roots)) == 64
    assert all(int(deg[r]) > 0 for r in roots)
    assert roots == gg.pick_roots(g, 64, seed=1)
