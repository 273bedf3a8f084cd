"""Pins of the oracle's weighted lists (subsections "Logarithmization of Edge
Weights" and "Accessing an Edge Weight": the weight right after the ID, at
one width omega = max(1, bl(largest weight))) and of its SSSP distances
(section "Considered Algorithms")."""

import heapq

import numpy as np
import pytest

import oracle as orc
from paper_2010_15879_amd import graphgen as gg


def weighted(n, wedges):
    """CSR plus per-entry weights from (u, v, w) triples (both directions)."""
    g = gg.csr_from_edges(n, [(u, v) for u, v, _ in wedges])
    off, col = g.numpy()
    wmap = {}
    for u, v, w in wedges:
        wmap[(u, v)] = wmap[(v, u)] = w
    wt = np.array([wmap[(u, int(col[i]))] for u in range(n) for i in range(off[u], off[u + 1])], np.uint32)
    return g, off, col, wt


def test_hand_stream_global():
    # n = 3: 0-1 weight 5, 0-2 weight 3; s = bl(2) = 2, omega = bl(5) = 3,
    # 5 bits per entry, entries in row order: (1,5) (2,3) | (0,5) | (0,3)
    # bits: 1 | 5<<2 = 21 at 0; 2 | 3<<2 = 14 at 5; 0 | 5<<2 = 20 at 10;
    # 0 | 3<<2 = 12 at 15 -> 21 + 14*32 + 20*1024 + 12*32768 = 414165
    g, off, col, wt = weighted(3, [(0, 1, 5), (0, 2, 3)])
    e = orc.Encoding(off, col, "global", "packed", weights=wt)
    assert e.s == 2 and e.omega == 3 and e.U == 20
    assert int(e.A[0]) == 414165
    np.testing.assert_array_equal(e.P, [0, 10, 15, 20])
    np.testing.assert_array_equal(e.neighbors(0), [1, 2])
    np.testing.assert_array_equal(e.weights_of(0), [5, 3])


def test_hand_stream_local():
    # same graph, local widths: w_0 = bl(2) = 2, w_1 = w_2 = 1 (bl(0) -> 1);
    # row 0 entries 5 bits each, rows 1 and 2 one entry of 1 + 3 = 4 bits
    # bits: 21 at 0; 14 at 5; 0 | 5<<1 = 10 at 10; 0 | 3<<1 = 6 at 14
    g, off, col, wt = weighted(3, [(0, 1, 5), (0, 2, 3)])
    e = orc.Encoding(off, col, "local", "packed", weights=wt)
    assert e.U == 18
    np.testing.assert_array_equal(e.P, [0, 10, 14, 18])
    assert int(e.A[0]) == 21 + 14 * 32 + 10 * 1024 + 6 * 16384


@pytest.mark.parametrize("ids", ["global", "local"])
def test_round_trip_and_size(ids):
    g = gg.kronecker(10, 8, seed=3)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 255, seed=2).numpy().astype(np.uint32)
    e = orc.Encoding(off, col, ids, "ef", weights=wt)
    assert e.omega == 8
    w = e.widths if ids == "local" else np.full(g.n, e.s)
    deg = off[1:] - off[:-1]
    assert e.U == int((deg * (w.astype(np.int64) + 8)).sum())
    for v in range(0, g.n, 7):
        np.testing.assert_array_equal(e.neighbors(v), col[off[v]:off[v + 1]])
        np.testing.assert_array_equal(e.weights_of(v), wt[off[v]:off[v + 1]])


def test_weights_symmetric_and_in_range():
    g = gg.kronecker(9, 8, seed=4)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 255, seed=9).numpy()
    assert wt.min() >= 1 and wt.max() <= 255
    pos = {}
    for u in range(g.n):
        for i in range(off[u], off[u + 1]):
            pos[(u, int(col[i]))] = wt[i]
    assert all(pos[(v, u)] == w for (u, v), w in pos.items())


def test_sssp_hand():
    # 0-1 (4), 0-2 (1), 2-1 (2), 1-3 (5), 2-3 (8), 4 isolated
    g, off, col, wt = weighted(5, [(0, 1, 4), (0, 2, 1), (2, 1, 2), (1, 3, 5), (2, 3, 8)])
    np.testing.assert_array_equal(orc.sssp(off, col, wt, 0), [0, 3, 1, 8, -1])
    np.testing.assert_array_equal(orc.sssp(off, col, wt, 3), [8, 5, 7, 0, -1])
    np.testing.assert_array_equal(orc.sssp(off, col, wt, 4), [-1, -1, -1, -1, 0])


def bellman_ford(n, off, col, wt, root):
    """Brute force: relax every edge n times."""
    INF = float("inf")
    d = [INF] * n
    d[root] = 0
    for _ in range(n):
        for u in range(n):
            if d[u] == INF:
                continue
            for i in range(off[u], off[u + 1]):
                if d[u] + int(wt[i]) < d[int(col[i])]:
                    d[int(col[i])] = d[u] + int(wt[i])
    return [-1 if x == INF else x for x in d]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_sssp_brute_force(seed):
    g = gg.random_graph(40, 0.1, seed=seed)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 20, seed=seed).numpy().astype(np.uint32)
    for root in (0, 7, 39):
        np.testing.assert_array_equal(orc.sssp(off, col, wt, root), bellman_ford(g.n, off, col, wt, root))


def test_sssp_unit_weights_are_bfs_depths():
    g = gg.kronecker(11, 8, seed=6)
    off, col = g.numpy()
    wt = np.ones(col.size, np.uint32)
    root = gg.pick_roots(g, 1, seed=2)[0]
    depth, _ = orc.bfs(off, col, root)
    np.testing.assert_array_equal(orc.sssp(off, col, wt, root), depth)


def test_sssp_triangle_inequality_and_tightness():
    """Distances satisfy d(v) <= d(u) + w(u, v) on every edge, and every
    reached vertex but the root has an edge where equality holds."""
    g = gg.erdos_renyi(11, 8, seed=7)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 255, seed=3).numpy().astype(np.int64)
    d = orc.sssp(off, col, wt.astype(np.uint32), 5)
    tight = np.zeros(g.n, bool)
    for u in range(g.n):
        if d[u] < 0:
            continue
        for i in range(off[u], off[u + 1]):
            v = int(col[i])
            assert d[v] >= 0 and d[v] <= d[u] + wt[i]
            tight[v] |= d[v] == d[u] + wt[i]
    reached = d >= 0
    reached[5] = False
    assert tight[reached].all()


def test_sssp_against_heapq():
    """A second Dijkstra written with Python's heapq on a larger graph."""
    g = gg.kronecker(12, 16, seed=8)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 255, seed=4).numpy()
    root = gg.pick_roots(g, 1, seed=5)[0]
    dist = {root: 0}
    pq = [(0, root)]
    done = set()
    while pq:
        d, u = heapq.heappop(pq)
        if u in done:
            continue
        done.add(u)
        for i in range(off[u], off[u + 1]):
            v, nd = int(col[i]), d + int(wt[i])
            if v not in dist or nd < dist[v]:
                dist[v] = nd
                heapq.heappush(pq, (nd, v))
    expect = np.full(g.n, -1, np.int64)
    for v, d in dist.items():
        expect[v] = d
    np.testing.assert_array_equal(orc.sssp(off, col, wt.astype(np.uint32), root), expect)


def test_relabeled_weights_follow_their_edges():
    """After the degree relabeling every stored entry still carries the weight
    of the edge it stands for, and the distances from a root are the same
    under the relabeling (mapped through it)."""
    g = gg.kronecker(10, 8, seed=5)
    off, col = g.numpy()
    wt = gg.edge_weights(g, 255, seed=7).numpy().astype(np.uint32)
    e = orc.Encoding(off, col, "local", "packed", True, weights=wt)
    w_of = {}
    for u in range(g.n):
        for i in range(off[u], off[u + 1]):
            w_of[(u, int(col[i]))] = int(wt[i])
    for r in range(0, g.n, 17):
        ids, ws = e.neighbors(r), e.weights_of(r)
        for c, w in zip(ids, ws):
            assert w_of[(int(e.perm[r]), int(e.perm[c]))] == int(w)
    root = gg.pick_roots(g, 1, seed=3)[0]
    d = orc.sssp(off, col, wt, root)
    d_new = orc.sssp(e.off, e.col, e.weights, int(e.inv[root]))
    np.testing.assert_array_equal(d_new[e.inv], d)
