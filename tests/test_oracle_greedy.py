"""Pins of the oracle's greedy relabeling heuristic (subsection "Adding
Integer Linear Programming", its listing of a greedy heuristic for vertex
relabeling): vertices in increasing order of degree (ties by ID) hand the
next unused label to each unlabeled neighbor, in list order; vertices that
never receive one take the remaining labels in ID order.  The expected
labels below are worked out by hand from that description."""

import numpy as np
import pytest

import oracle as orc
from paper_2010_15879_amd import graphgen as gg

# (n, undirected edges, inv by hand: inv[v] = new label of v)
HAND = {
    # degrees 1,2,2,1 -> order 0,3,1,2.  0 labels 1:0; 3 labels 2:1;
    # 1 labels 0:2; 2 labels 3:3
    "path4": (4, [(0, 1), (1, 2), (2, 3)], [2, 0, 1, 3]),
    # degrees 1,1,0 -> order 2,0,1.  0 labels 1:0; 1 labels 0:1; 2 is left
    "edge_plus_isolated": (3, [(0, 1)], [1, 0, 2]),
    # leaves first: 1 labels the center 0:0; the center labels 1..4 in order
    "star5": (5, [(0, i) for i in range(1, 5)], [0, 1, 2, 3, 4]),
    # degrees 2,2,3,2,1 -> order 4,0,1,3,2.  4 labels 3:0; 0 labels 1:1, 2:2;
    # 1 labels 0:3; 3 labels 4:4
    "triangle_tail": (5, [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4)], [3, 1, 2, 0, 4]),
    # equal degrees keep ID order: 0 labels 1:0, 4:1; 1 labels 0:2, 2:3;
    # 2 labels 3:4
    "cycle5": (5, [(i, (i + 1) % 5) for i in range(5)], [2, 0, 3, 4, 1]),
}


@pytest.mark.parametrize("case", sorted(HAND))
def test_greedy_hand_examples(case):
    n, edges, inv_hand = HAND[case]
    off, col = gg.csr_from_edges(n, edges).numpy()
    perm, inv = orc.greedy_permutation(off, col)
    np.testing.assert_array_equal(inv, np.array(inv_hand, np.uint32))
    np.testing.assert_array_equal(perm[inv], np.arange(n, dtype=np.uint32))


@pytest.mark.parametrize("seed", [1, 2])
def test_greedy_invariants(seed):
    g = gg.kronecker(9, 8, seed=seed)
    off, col = g.numpy()
    n = g.n
    perm, inv = orc.greedy_permutation(off, col)
    # a permutation, perm and inv inverse to each other
    np.testing.assert_array_equal(np.sort(perm), np.arange(n, dtype=np.uint32))
    np.testing.assert_array_equal(perm[inv], np.arange(n, dtype=np.uint32))
    # edgeless vertices take the last labels, in ID order
    deg = np.diff(off.astype(np.int64))
    iso = np.nonzero(deg == 0)[0]
    assert np.array_equal(perm[n - iso.size:], iso.astype(np.uint32))
    # the first vertex with edges in (degree, ID) order hands out the first
    # labels, to its neighbors in list order (edgeless vertices come before
    # it but label nobody)
    nz = np.nonzero(deg > 0)[0]
    v0 = int(nz[np.lexsort((nz, deg[nz]))[0]])
    first = col[off[v0]:off[v0 + 1]]
    assert first.size > 0
    np.testing.assert_array_equal(inv[first], np.arange(first.size, dtype=np.uint32))
