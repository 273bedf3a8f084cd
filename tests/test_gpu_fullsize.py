"""Parity at full size, in the launch configuration the benchmark times.

Kronecker scale 24 (DM relabel, local widths, Elias-Fano offsets) and
Erdos-Renyi scale 26 (global widths, packed offsets), each also on the plain
uint32 CSR.  The oracle computes whole arrays (permutation, widths, bit
starts, Elias-Fano arrays, packed offsets), sampled rows of the packed lists
bit by bit, four whole BFS trees per layout (rows of the 64-root call the
benchmark times, against the oracle's level-synchronous BFS) and the whole
20-iteration PageRank vector (against the oracle's all-core PageRank, which
equals its one-thread loop bit for bit)."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


def host_csr(g):
    """Host copies in the oracle's element types (no per-call conversions)."""
    off, col = g.numpy()
    return off.astype(np.uint64), col.view(np.uint32)


def check_trees_and_pagerank(lgmod, h, g, off, col, labels, what):
    """Four whole BFS trees out of the benchmark's 64-root call (the call it
    times) and the whole 20-iteration PageRank vector."""
    roots = gg.pick_roots(g, 64, seed=1)
    pick = [0, 21, 42, 63]
    print(f"[fullsize] {what}: BFS from {len(roots)} roots, rows {pick} checked", flush=True)
    depth, parent = lgmod.bfs(h, roots)
    depth, parent = depth[pick].cpu().numpy(), parent[pick].cpu().numpy()
    for i, k in enumerate(pick):
        r = roots[k]
        d0, p0 = orc.bfs_levels(off, col, r, labels=labels)
        np.testing.assert_array_equal(depth[i], d0, err_msg=f"{what} root {r}")
        np.testing.assert_array_equal(parent[i], p0, err_msg=f"{what} root {r}")
    print(f"[fullsize] {what}: PageRank, 20 iterations", flush=True)
    pr = lgmod.pagerank(h, 0.85, 20).cpu().numpy().astype(np.float64)
    return pr


def pagerank20(off, col):
    """The oracle's 20-iteration FP64 PageRank (all host cores)."""
    return orc.pagerank_par(off, col, 0.85, 20)


def check_sampled_rows(A, P, W, F, s, rows, expect_row):
    """Every bit of the sampled rows of the packed stream, read bit by bit."""
    for x in rows:
        want = expect_row(x)
        w = orc.get_bits(W, x * F, F) if W is not None else s
        got = orc.decode_list(A, int(P[x]), want.size, w)
        np.testing.assert_array_equal(got, want, err_msg=f"row {x}")


def test_kronecker24_local_ef_relabeled(lgmod):
    print("[fullsize] kronecker s24: generate", flush=True)
    g = gg.kronecker(24, 16, seed=1, device="cuda")
    off, col = host_csr(g)
    n = g.n
    print("[fullsize] kronecker s24: encode", flush=True)
    h = lgmod.encode(g.row_offsets, g.col, n, ids="local", offsets="succinct", relabel=True)
    info = h.info()
    # permutation: the whole array
    perm, inv = orc.dm_permutation(off)
    np.testing.assert_array_equal(h.export("perm"), perm)
    np.testing.assert_array_equal(h.export("inv"), inv)
    # widths, bit starts, width table and the Elias-Fano arrays: whole arrays
    w, d2 = orc.relabeled_local_widths(off, col, perm, inv)
    off2 = np.zeros(n + 1, dtype=np.uint64)
    off2[1:] = np.cumsum(d2)
    P = orc.bit_starts(off2, w, 0)
    assert info["adj_bits"] == int(P[-1])
    F = orc.width_field_bits(n)
    W = h.export("widths")
    np.testing.assert_array_equal(W, orc.pack_fixed(w.astype(np.uint64), F))
    ef = orc.EF(P, int(P[-1]))
    np.testing.assert_array_equal(h.export("ef_low"), ef.low)
    np.testing.assert_array_equal(h.export("ef_high"), ef.high)
    np.testing.assert_array_equal(h.export("ef_rank"), ef.rank_sb)
    np.testing.assert_array_equal(h.export("ef_select"), ef.sel)
    # the packed lists: sampled rows (hubs, middle, last non-empty), every bit
    A = h.export("adj")
    assert A.size == (int(P[-1]) + 63) // 64 + 1 and int(A[-1]) == 0
    rng = np.random.default_rng(11)
    nonempty = int(np.count_nonzero(d2))
    rows = sorted(set([0, 1, 2, 63, 64, 65, nonempty - 1] + rng.integers(0, nonempty, 300).tolist()))
    check_sampled_rows(A, P, W, F, 0, rows, lambda x: orc.relabel_row(off, col, perm, inv, x))
    del A
    # BFS trees (depths and smallest-label parents) and the 20-iteration
    # PageRank vector, packed and plain (same labeling)
    pr64 = pagerank20(off, col)
    pr = check_trees_and_pagerank(lgmod, h, g, off, col, inv, "kronecker s24 packed")
    assert np.abs(pr - pr64).sum() <= 1e-5
    # the first iterations too (the error grows with the iterations)
    pr1 = lgmod.pagerank(h, 0.85, 1).cpu().numpy().astype(np.float64)
    assert np.abs(pr1 - orc.pagerank_par(off, col, 0.85, 1)).sum() <= 1e-5
    h.free()
    hp = lgmod.encode(g.row_offsets, g.col, n, layout="plain", relabel=True)
    pr = check_trees_and_pagerank(lgmod, hp, g, off, col, inv, "kronecker s24 plain")
    assert np.abs(pr - pr64).sum() <= 1e-5
    hp.free()


def test_erdos_renyi26_packed_and_plain(lgmod):
    print("[fullsize] ER s26: generate", flush=True)
    g = gg.erdos_renyi(26, 16, seed=1, device="cuda")
    n, M = g.n, g.m
    assert M < (1 << 31) and orc.global_width(n) == 26
    print(f"[fullsize] ER s26: n={n} M={M}; encode packed", flush=True)
    h = lgmod.encode(g.row_offsets, g.col, n)
    info = h.info()
    assert info["s"] == 26 and info["adj_bits"] == 26 * M
    assert info["w_offset"] == orc.bitlen(M)
    off, col = host_csr(g)
    # packed offsets: the whole array
    np.testing.assert_array_equal(h.export("offsets"), orc.pack_fixed(off, orc.bitlen(M)))
    A = h.export("adj")
    assert A.size == (26 * M + 63) // 64 + 1 and int(A[-1]) == 0
    rng = np.random.default_rng(3)
    rows = sorted(set([0, n - 1] + rng.integers(0, n, 300).tolist()))
    P = orc.bit_starts(off, None, 26)
    check_sampled_rows(A, P, None, 0, 26, rows, lambda v: col[int(off[v]):int(off[v + 1])])
    del A
    print("[fullsize] ER s26: oracle PageRank, 20 iterations", flush=True)
    pr64 = pagerank20(off, col)
    pr = check_trees_and_pagerank(lgmod, h, g, off, col, None, "ER s26 packed")
    assert np.abs(pr - pr64).sum() <= 1e-5
    h.free()
    print("[fullsize] ER s26: plain CSR", flush=True)
    hp = lgmod.encode(g.row_offsets, g.col, n, layout="plain")
    pr = check_trees_and_pagerank(lgmod, hp, g, off, col, None, "ER s26 plain")
    assert np.abs(pr - pr64).sum() <= 1e-5
    pr1 = lgmod.pagerank(hp, 0.85, 1).cpu().numpy().astype(np.float64)
    assert np.abs(pr1 - orc.pagerank_par(off, col, 0.85, 1)).sum() <= 1e-5
    hp.free()


def test_kronecker24_greedy_relabel(lgmod):
    """The greedy relabeling at the benchmark's size: the whole permutation
    against the oracle's literal loop, the widths and bit starts it implies,
    and sampled rows of the packed lists."""
    print("[fullsize] kronecker s24 greedy: generate", flush=True)
    g = gg.kronecker(24, 16, seed=1, device="cuda")
    off, col = host_csr(g)
    n = g.n
    print("[fullsize] kronecker s24 greedy: encode", flush=True)
    h = lgmod.encode(g.row_offsets, g.col, n, ids="local", offsets="succinct", relabel="greedy")
    info = h.info()
    perm, inv = orc.greedy_permutation(off, col)
    np.testing.assert_array_equal(h.export("perm"), perm)
    np.testing.assert_array_equal(h.export("inv"), inv)
    w, d2 = orc.relabeled_local_widths(off, col, perm, inv)
    off2 = np.zeros(n + 1, dtype=np.uint64)
    off2[1:] = np.cumsum(d2)
    P = orc.bit_starts(off2, w, 0)
    assert info["adj_bits"] == int(P[-1])
    F = orc.width_field_bits(n)
    W = h.export("widths")
    np.testing.assert_array_equal(W, orc.pack_fixed(w.astype(np.uint64), F))
    A = h.export("adj")
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(8), rng.integers(0, n, size=64)])
    check_sampled_rows(A, P, W, F, 0, rows, lambda x: orc.relabel_row(off, col, perm, inv, int(x)))
    h.free()


def test_kronecker24_gap_and_dmd(lgmod):
    """Fixed-size gap lists and Varint differences (DMd), both after the
    degree relabeling, at the benchmark's size: one whole BFS tree, the first
    PageRank iteration, and sampled decoded lists against the oracle."""
    print("[fullsize] kronecker s24 gap/DMd: generate", flush=True)
    g = gg.kronecker(24, 16, seed=1, device="cuda")
    off, col = host_csr(g)
    root = gg.pick_roots(g, 1, seed=2)[0]
    print("[fullsize] kronecker s24 gap/DMd: oracle BFS and PageRank", flush=True)
    d0, p0 = orc.bfs(off, col, root, relabeled=True)
    pr64 = orc.pagerank(off, col, 0.85, 1)
    rng = np.random.default_rng(12)
    vs = rng.integers(0, g.n, 300).astype(np.int32)
    for ids in ("local-gap", "varint-diff"):
        print(f"[fullsize] kronecker s24 {ids}: encode, BFS, PageRank, decode", flush=True)
        h = lgmod.encode(g.row_offsets, g.col, g.n, ids=ids, offsets="succinct", relabel=True)
        depth, parent = lgmod.bfs(h, [root])
        np.testing.assert_array_equal(depth[0].cpu().numpy(), d0)
        np.testing.assert_array_equal(parent[0].cpu().numpy(), p0)
        pr = lgmod.pagerank(h, 0.85, 1).cpu().numpy().astype(np.float64)
        assert np.abs(pr - pr64).sum() <= 1e-5
        o_off, o_ids = lgmod.decode_neighbors(h, torch.from_numpy(vs).cuda(), "sorted")
        o_off, o_ids = o_off.cpu().numpy(), o_ids.cpu().numpy()
        for i, v in enumerate(vs):
            np.testing.assert_array_equal(o_ids[o_off[i]:o_off[i + 1]], col[off[v]:off[v + 1]])
        h.free()


def test_kronecker22_weighted_sssp(lgmod):
    """Weighted SSSP at Kronecker scale 22 (weights uniform in [1, 255]):
    the whole distance array against the oracle's Dijkstra, packed local IDs
    with Elias-Fano offsets (unrelabeled, and after the degree and greedy
    relabelings, which search in label space and map back) and the plain
    CSR."""
    print("[fullsize] kronecker s22 sssp: generate", flush=True)
    g = gg.kronecker(22, 16, seed=3, device="cuda")
    wt = gg.edge_weights(g, 255, seed=1)
    off, col = host_csr(g)
    root = gg.pick_roots(g, 1, seed=4)[0]
    print("[fullsize] kronecker s22 sssp: oracle", flush=True)
    expect = orc.sssp(off, col, wt.cpu().numpy().astype(np.uint32), root)
    for kw in (dict(ids="local", offsets="succinct"), dict(layout="plain"),
               dict(ids="local", offsets="succinct", relabel=True),
               dict(ids="local", offsets="succinct", relabel="greedy")):
        print(f"[fullsize] kronecker s22 sssp: {kw}", flush=True)
        h = lgmod.encode(g.row_offsets, g.col, g.n, weights=wt, **kw)
        np.testing.assert_array_equal(lgmod.sssp(h, root).cpu().numpy(), expect)
        h.free()
