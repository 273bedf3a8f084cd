"""Pins of the oracle's relabeling, BFS and PageRank.

Paper passages: "Incorporating Degree-Minimizing (DM)" (higher degree gets
a lower label) and "Considered Algorithms" (BFS; PageRank without atomics).
BFS is pinned against Floyd-Warshall / all-pairs brute force, an exhaustive
sweep of every graph on 5 labelled vertices, networkx and scipy; PageRank
against dense power iteration with the Google matrix, closed forms and the
dominant eigenvector."""

import itertools

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle as orc
from paper_2010_15879_amd import graphgen as gg


def csr_of(n, edges):
    g = gg.csr_from_edges(n, edges)
    return g.numpy()


# -- degree-minimizing relabel ----------------------------------------

def test_dm_permutation_properties():
    g = gg.kronecker(10, 8, seed=4)
    off, col = g.numpy()
    perm, inv = orc.dm_permutation(off)
    n = g.n
    assert sorted(perm.tolist()) == list(range(n))                     # bijection
    np.testing.assert_array_equal(inv[perm], np.arange(n))
    deg = np.diff(off.astype(np.int64))
    dn = deg[perm]
    assert np.all(dn[:-1] >= dn[1:])                                   # non-increasing
    ties = dn[:-1] == dn[1:]
    assert np.all(perm[:-1][ties] < perm[1:][ties])                    # ties keep original order
    # independent formulation: numpy's stable lexsort on (-degree, id)
    np.testing.assert_array_equal(perm, np.lexsort((np.arange(n), -deg)))


def test_dm_hand_example():
    # degrees: 0:1 1:3 2:2 3:2 4:0  -> order by (deg desc, id): 1, 2, 3, 0, 4
    off, col = csr_of(5, [(0, 1), (1, 2), (1, 3), (2, 3)])
    perm, inv = orc.dm_permutation(off)
    assert perm.tolist() == [1, 2, 3, 0, 4]
    assert inv.tolist() == [3, 0, 1, 2, 4]
    off2, col2 = orc.relabel(off, col, perm, inv)
    # new graph edges: 0-1 (1-2), 0-2 (1-3), 0-3 (1-0), 1-2 (2-3)
    assert off2.tolist() == [0, 3, 5, 7, 8, 8]
    assert col2.tolist() == [1, 2, 3, 0, 2, 0, 1, 0]


def test_relabel_roundtrip():
    g = gg.kronecker(9, 8, seed=6)
    off, col = g.numpy()
    perm, inv = orc.dm_permutation(off)
    off2, col2 = orc.relabel(off, col, perm, inv)
    # lists sorted, graph isomorphic, mapping back reproduces the input CSR
    for x in range(g.n):
        lst = col2[off2[x]:off2[x + 1]]
        assert np.all(np.diff(lst.astype(np.int64)) > 0)
        back = np.sort(perm[lst])
        v = perm[x]
        np.testing.assert_array_equal(back, col[off[v]:off[v + 1]])
        if x % 37 == 0:
            np.testing.assert_array_equal(orc.relabel_row(off, col, perm, inv, x), lst)


# -- BFS --------------------------------------------------------------

def allpairs_hops(n, off, col):
    """Floyd-Warshall on unit weights."""
    INF = 10 ** 9
    D = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for v in range(n):
        for u in col[off[v]:off[v + 1]]:
            D[v, u] = 1
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= INF] = -1
    return D


def check_parents(n, off, col, root, depth, parent, labels=None):
    lab = np.arange(n) if labels is None else labels
    for v in range(n):
        if depth[v] < 0:
            assert parent[v] == -1
        elif v == root:
            assert parent[v] == root
        else:
            p = parent[v]
            assert p in col[off[v]:off[v + 1]]                 # tree edge exists
            assert depth[p] == depth[v] - 1
            ups = [u for u in col[off[v]:off[v + 1]] if depth[u] == depth[v] - 1]
            assert lab[p] == min(lab[u] for u in ups)          # smallest label


def test_bfs_golden(golden):
    fx = golden("bfs_small.txt")
    e = fx["edges"]
    off, col = csr_of(fx["n"][0], list(zip(e[0::2], e[1::2])))
    d, p = orc.bfs(off, col, fx["root"][0])
    assert d.tolist() == fx["depth"]
    assert p.tolist() == fx["parent"]
    d2, p2 = orc.bfs(off, col, fx["root"][0], max_depth=2)
    assert d2.tolist() == fx["depth_k2"]
    assert p2.tolist() == fx["parent_k2"]


@pytest.mark.parametrize("seed", range(6))
def test_bfs_vs_floyd_warshall(seed):
    n = [1, 2, 17, 33, 64, 64][seed]
    g = gg.random_graph(n, [0.5, 0.5, 0.15, 0.08, 0.05, 0.1][seed], seed=seed)
    off, col = g.numpy()
    D = allpairs_hops(n, off, col)
    for root in range(n):
        d, p = orc.bfs(off, col, root)
        np.testing.assert_array_equal(d, D[root])
        check_parents(n, off, col, root, d, p)


def test_bfs_exhaustive_five_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        off, col = csr_of(5, edges)
        D = allpairs_hops(5, off, col)
        for root in range(5):
            d, p = orc.bfs(off, col, root)
            assert d.tolist() == D[root].tolist()
            for v in range(5):
                if d[v] > 0:
                    ups = [u for u in col[off[v]:off[v + 1]] if d[u] == d[v] - 1]
                    assert p[v] == min(ups)


def test_bfs_vs_networkx_and_scipy():
    g = gg.kronecker(11, 4, seed=8)
    off, col = g.numpy()
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(off.astype(np.int64)))
    G.add_edges_from(zip(src.tolist(), col.tolist()))
    A = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), off.astype(np.int64)), shape=(g.n, g.n))
    ncomp, comp = csg.connected_components(A, directed=False)
    for root in gg.pick_roots(g, 4, seed=3):
        d, p = orc.bfs(off, col, root)
        want = nx.single_source_shortest_path_length(G, root)
        assert {v: int(d[v]) for v in range(g.n) if d[v] >= 0} == want
        np.testing.assert_array_equal(d >= 0, comp == comp[root])       # reached set = component
        hop = csg.shortest_path(A, unweighted=True, indices=root)
        np.testing.assert_array_equal(np.where(np.isinf(hop), -1, hop).astype(np.int32), d)
        check_parents(g.n, off, col, root, d, p)
        # every edge between reached vertices spans at most one level
        reached = d[src] >= 0
        assert np.all(np.abs(d[src][reached] - d[col][reached]) <= 1)


def test_bfs_k_hop_is_truncation():
    g = gg.kronecker(10, 8, seed=12)
    off, col = g.numpy()
    root = gg.pick_roots(g, 1)[0]
    d, p = orc.bfs(off, col, root)
    for k in [0, 1, 2, 3]:
        dk, pk = orc.bfs(off, col, root, max_depth=k)
        keep = (d >= 0) & (d <= k)
        np.testing.assert_array_equal(dk, np.where(keep, d, -1))
        np.testing.assert_array_equal(pk, np.where(keep, p, -1))


def test_bfs_relabeled_parents():
    g = gg.kronecker(10, 8, seed=13)
    off, col = g.numpy()
    perm, inv = orc.dm_permutation(off)
    off2, col2 = orc.relabel(off, col, perm, inv)
    for root in gg.pick_roots(g, 3, seed=2):
        d, p = orc.bfs(off, col, root, relabeled=True)
        d0, _ = orc.bfs(off, col, root)
        np.testing.assert_array_equal(d, d0)                  # depths are label-free
        check_parents(g.n, off, col, root, d, p, labels=inv)  # smallest new label
        # the same tree computed on the relabeled CSR, mapped back
        dn, pn = orc.bfs(off2, col2, int(inv[root]))
        np.testing.assert_array_equal(dn[inv], d)
        np.testing.assert_array_equal(np.where(pn[inv] < 0, -1, perm.astype(np.int64)[np.maximum(pn[inv], 0)]), p)


def test_bfs_isolated_root_and_singleton():
    off, col = csr_of(4, [(1, 2)])
    d, p = orc.bfs(off, col, 0)
    assert d.tolist() == [0, -1, -1, -1] and p.tolist() == [0, -1, -1, -1]
    off, col = csr_of(1, [])
    d, p = orc.bfs(off, col, 0)
    assert d.tolist() == [0] and p.tolist() == [0]


# -- PageRank ---------------------------------------------------------

def google_power_iteration(n, off, col, alpha, iters):
    """Dense power iteration x <- G x with the Google matrix
    G = alpha (A D^-1 + (1/n) 1 z^T) + (1 - alpha)/n 1 1^T, where z marks
    vertices without edges."""
    A = np.zeros((n, n))
    for v in range(n):
        for u in col[off[v]:off[v + 1]]:
            A[v, u] = 1.0
    deg = A.sum(axis=0)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = A[:, nz] / deg[nz]
    M[:, ~nz] = 1.0 / n
    G = alpha * M + (1 - alpha) / n
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = G @ x
    return x, G


@pytest.mark.parametrize("seed", range(5))
def test_pagerank_vs_dense_google_matrix(seed):
    n = [2, 9, 31, 64, 64][seed]
    g = gg.random_graph(n, [1.0, 0.3, 0.1, 0.05, 0.02][seed], seed=seed + 20)
    off, col = g.numpy()
    pr = orc.pagerank(off, col, 0.85, 20)
    x, _ = google_power_iteration(n, off, col, 0.85, 20)
    np.testing.assert_allclose(pr, x, rtol=0, atol=1e-12)
    assert abs(pr.sum() - 1.0) < 1e-12


def test_pagerank_converged_is_dominant_eigenvector():
    g = gg.random_graph(40, 0.1, seed=33)
    off, col = g.numpy()
    pr = orc.pagerank(off, col, 0.85, 300)
    _, G = google_power_iteration(40, off, col, 0.85, 0)
    w, V = np.linalg.eig(G)
    k = int(np.argmax(np.abs(w)))
    assert abs(w[k] - 1.0) < 1e-10
    vec = np.real(V[:, k])
    vec = vec / vec.sum()
    np.testing.assert_allclose(pr, vec, rtol=0, atol=1e-12)


def test_pagerank_star_fixed_point(golden):
    fx = golden("pagerank_star.txt")
    off, col = csr_of(5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    pr = orc.pagerank(off, col, fx["alpha"][0], 400)
    assert abs(pr[0] - fx["centre"][0]) < 1e-14
    np.testing.assert_allclose(pr[1:], fx["leaf"][0], rtol=0, atol=1e-14)


def test_pagerank_regular_graph_stays_uniform():
    n = 12
    off, col = csr_of(n, [(i, (i + 1) % n) for i in range(n)] + [(i, (i + 5) % n) for i in range(n)])
    assert len(set(np.diff(off.astype(np.int64)).tolist())) == 1
    for t in [1, 2, 20]:
        np.testing.assert_allclose(orc.pagerank(off, col, 0.85, t), 1.0 / n, rtol=0, atol=1e-15)


def test_pagerank_isolated_vertex_closed_form():
    # vertex 3 has no edges: PR_{t+1}(3) = (1-a)/n + a D_t / n, D_t = PR_t(3)
    off, col = csr_of(4, [(0, 1), (1, 2), (0, 2)])
    a, n = 0.85, 4
    x = 1.0 / n
    for t in range(1, 8):
        x = (1 - a) / n + a * x / n
        assert abs(orc.pagerank(off, col, a, t)[3] - x) < 1e-15


def test_pagerank_alpha_one_random_walk():
    # a = 1 on a connected non-bipartite graph without isolated vertices
    # converges to the random walk's stationary distribution d_v / M
    g = gg.random_graph(30, 0.25, seed=5)
    off, col = g.numpy()
    A = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), off.astype(np.int64)), shape=(30, 30))
    assert csg.connected_components(A, directed=False)[0] == 1
    assert not nx.is_bipartite(nx.from_scipy_sparse_array(A))
    pr = orc.pagerank(off, col, 1.0, 2000)
    np.testing.assert_allclose(pr, np.diff(off.astype(np.int64)) / col.size, rtol=0, atol=1e-12)


def test_relabeled_widths_match_relabeled_csr():
    g = gg.kronecker(10, 8, seed=21)
    off, col = g.numpy()
    perm, inv = orc.dm_permutation(off)
    off2, col2 = orc.relabel(off, col, perm, inv)
    w, d = orc.relabeled_local_widths(off, col, perm, inv)
    np.testing.assert_array_equal(w, orc.local_widths(off2, col2))
    np.testing.assert_array_equal(d, np.diff(off2.astype(np.uint64)))
