"""Pins of the oracle's all-core PageRank and level-synchronous BFS.

They compute the same results as the one-thread oracle functions on every
host core (they exist so that the full-size parity tests and the CPU
baseline can afford the oracle).  Paper passage: "Considered Algorithms"
(BFS, PageRank without atomics).  Each is pinned on its own -- BFS against
Floyd-Warshall, an exhaustive sweep of every graph on 5 labelled vertices,
networkx and scipy; PageRank against dense power iteration with the Google
matrix and closed forms -- and held bit for bit to the one-thread
functions on Kronecker and Erdos-Renyi graphs, with several thread
counts."""

import itertools

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle as orc
from paper_2010_15879_amd import graphgen as gg
from test_oracle_algorithms import allpairs_hops, check_parents, csr_of, google_power_iteration

THREADS = [1, 3, 8]


# -- level-synchronous BFS ------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_bfs_levels_vs_floyd_warshall(seed):
    n = [1, 2, 17, 33, 64, 64][seed]
    g = gg.random_graph(n, [0.5, 0.5, 0.15, 0.08, 0.05, 0.1][seed], seed=seed)
    off, col = g.numpy()
    D = allpairs_hops(n, off, col)
    for root in range(n):
        d, p = orc.bfs_levels(off, col, root, threads=THREADS[root % 3])
        np.testing.assert_array_equal(d, D[root])
        check_parents(n, off, col, root, d, p)


def test_bfs_levels_exhaustive_five_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        off, col = csr_of(5, edges)
        D = allpairs_hops(5, off, col)
        for root in range(5):
            d, p = orc.bfs_levels(off, col, root, threads=2)
            assert d.tolist() == D[root].tolist()
            for v in range(5):
                if d[v] > 0:
                    ups = [u for u in col[off[v]:off[v + 1]] if d[u] == d[v] - 1]
                    assert p[v] == min(ups)


def test_bfs_levels_vs_networkx_and_scipy():
    g = gg.kronecker(11, 4, seed=8)
    off, col = g.numpy()
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(off.astype(np.int64)))
    G.add_edges_from(zip(src.tolist(), col.tolist()))
    A = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), off.astype(np.int64)), shape=(g.n, g.n))
    for root in gg.pick_roots(g, 4, seed=3):
        d, p = orc.bfs_levels(off, col, root, threads=4)
        want = nx.single_source_shortest_path_length(G, root)
        assert {v: int(d[v]) for v in range(g.n) if d[v] >= 0} == want
        hop = csg.shortest_path(A, unweighted=True, indices=root)
        np.testing.assert_array_equal(np.where(np.isinf(hop), -1, hop).astype(np.int32), d)
        check_parents(g.n, off, col, root, d, p)


@pytest.mark.parametrize("gen", ["kronecker", "er"])
def test_bfs_levels_equals_fifo(gen):
    """Whole depth and parent arrays equal the FIFO search's, with IDs and
    with the degree permutation's labels as the parent rule, for full and
    k-hop searches."""
    g = (gg.kronecker if gen == "kronecker" else gg.erdos_renyi)(14, 16, seed=5)
    off, col = g.numpy()
    perm, inv = orc.dm_permutation(off)
    for i, root in enumerate(gg.pick_roots(g, 4, seed=1)):
        for k in (-1, 0, 1, 2):
            d0, p0 = orc.bfs(off, col, root, max_depth=k)
            d1, p1 = orc.bfs_levels(off, col, root, max_depth=k, threads=THREADS[i % 3])
            np.testing.assert_array_equal(d1, d0)
            np.testing.assert_array_equal(p1, p0)
        d0, p0 = orc.bfs(off, col, root, relabeled=True)
        d1, p1 = orc.bfs_levels(off, col, root, labels=inv, threads=8)
        np.testing.assert_array_equal(d1, d0)
        np.testing.assert_array_equal(p1, p0)


def test_bfs_levels_isolated_root_and_singleton():
    off, col = csr_of(4, [(1, 2)])
    d, p = orc.bfs_levels(off, col, 0)
    assert d.tolist() == [0, -1, -1, -1] and p.tolist() == [0, -1, -1, -1]
    off, col = csr_of(1, [])
    d, p = orc.bfs_levels(off, col, 0)
    assert d.tolist() == [0] and p.tolist() == [0]


# -- all-core PageRank ----------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_pagerank_par_vs_dense_google_matrix(seed):
    n = [2, 9, 31, 64, 64][seed]
    g = gg.random_graph(n, [1.0, 0.3, 0.1, 0.05, 0.02][seed], seed=seed + 20)
    off, col = g.numpy()
    pr = orc.pagerank_par(off, col, 0.85, 20, threads=THREADS[seed % 3])
    x, _ = google_power_iteration(n, off, col, 0.85, 20)
    np.testing.assert_allclose(pr, x, rtol=0, atol=1e-12)
    assert abs(pr.sum() - 1.0) < 1e-12


def test_pagerank_par_closed_forms(golden):
    fx = golden("pagerank_star.txt")
    off, col = csr_of(5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    pr = orc.pagerank_par(off, col, fx["alpha"][0], 400, threads=3)
    assert abs(pr[0] - fx["centre"][0]) < 1e-14
    np.testing.assert_allclose(pr[1:], fx["leaf"][0], rtol=0, atol=1e-14)
    # an isolated vertex: PR_{t+1}(3) = (1-a)/n + a PR_t(3)/n
    off, col = csr_of(4, [(0, 1), (1, 2), (0, 2)])
    a, n, x = 0.85, 4, 0.25
    for t in range(1, 8):
        x = (1 - a) / n + a * x / n
        assert abs(orc.pagerank_par(off, col, a, t, threads=2)[3] - x) < 1e-15


@pytest.mark.parametrize("gen", ["kronecker", "er"])
def test_pagerank_par_bit_identical(gen):
    g = (gg.kronecker if gen == "kronecker" else gg.erdos_renyi)(14, 16, seed=7)
    off, col = g.numpy()
    for iters in (1, 2, 20):
        a = orc.pagerank(off, col, 0.85, iters)
        for t in THREADS:
            b = orc.pagerank_par(off, col, 0.85, iters, threads=t)
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (iters, t)
