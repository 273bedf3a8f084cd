"""lg_bfs with many roots runs batches of at least 16 of them as one
multi-source traversal and the rest a few at a time on internal streams:
every row must equal the result of a call with that root alone, whichever
path took it, and work on the caller's stream must be ordered around the
call."""

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


def small_graph(name):
    """A skewed graph (many vertices over the heavy-degree threshold) and an
    even-degree one: the multi-source resolve picks its grid by that."""
    if name == "kron13":
        return gg.kronecker(13, 16, seed=5, device="cuda")
    return gg.erdos_renyi(13, 8, seed=3, device="cuda")


@pytest.mark.parametrize("graph", ["kron13", "er13"])
@pytest.mark.parametrize("count", [9, 37, 70])
@pytest.mark.parametrize("kw", [dict(), dict(ids="local", offsets="succinct", relabel=True),
                                dict(layout="plain", relabel=True)])
@pytest.mark.parametrize("max_depth", [-1, 2])
def test_many_roots_equal_one_at_a_time(lgmod, graph, count, kw, max_depth):
    """9 roots: lanes only; 37: one multi-source batch; 70: a batch of 64 and
    six roots on the lanes."""
    g = small_graph(graph)
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    roots = gg.pick_roots(g, count, seed=2)
    d_all, p_all = lgmod.bfs(h, roots, max_depth=max_depth)
    for i, r in enumerate(roots):
        d1, p1 = lgmod.bfs(h, [r], max_depth=max_depth)
        assert torch.equal(d_all[i], d1[0]) and torch.equal(p_all[i], p1[0]), (i, r)
    off, col = g.numpy()
    for i in sorted({0, len(roots) // 2, len(roots) - 1}):
        d0, p0 = orc.bfs(off.astype(np.uint64), col.view(np.uint32), roots[i], max_depth=max_depth,
                         relabeled=bool(kw.get("relabel")))
        np.testing.assert_array_equal(d_all[i].cpu().numpy(), d0)
        np.testing.assert_array_equal(p_all[i].cpu().numpy(), p0)
    h.free()


@pytest.mark.parametrize("count", [9, 40])
def test_stream_order_around_the_call(lgmod, count):
    """Outputs written on the caller's stream before the call are overwritten by
    it, and a kernel queued after the call sees the final rows."""
    g = gg.kronecker(12, 16, seed=9, device="cuda")
    h = lgmod.encode(g.row_offsets, g.col, g.n)
    roots = gg.pick_roots(g, count, seed=3)
    ref, _ = lgmod.bfs(h, roots)
    torch.cuda.synchronize()
    for _ in range(3):
        depth = torch.empty((len(roots), g.n), dtype=torch.int32, device="cuda")
        parent = torch.empty_like(depth)
        depth.fill_(123)          # queued before: must not land after the BFS writes
        lgmod.bfs(h, roots, depth_out=depth, parent_out=parent)
        total = depth.sum()       # queued after: must see the finished rows
        assert torch.equal(depth, ref)
        assert int(total) == int(ref.sum())
    h.free()


@pytest.mark.parametrize("graph", ["kron12", "er12"])
@pytest.mark.parametrize("kw", [dict(), dict(ids="local", offsets="succinct", relabel=True),
                                dict(layout="plain")])
def test_repeated_and_edgeless_roots_over_two_batches(lgmod, graph, kw):
    """About 100 roots (two multi-source batches back to back, sharing the
    masks), with a root given three times and edgeless roots among them:
    every row equals the call with that root alone, and an edgeless root's
    row holds only itself."""
    g = gg.kronecker(12, 8, seed=7, device="cuda") if graph == "kron12" else \
        gg.erdos_renyi(12, 2, seed=7, device="cuda")
    iso = torch.nonzero(g.degrees() == 0).flatten()[:3].tolist()
    assert len(iso) == 3
    base = gg.pick_roots(g, 95, seed=4)
    roots = base[:30] + [base[3], base[3]] + iso + base[30:]
    assert len(roots) > 64 + 32
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    d_all, p_all = lgmod.bfs(h, roots)
    for i, r in enumerate(roots):
        d1, p1 = lgmod.bfs(h, [r])
        assert torch.equal(d_all[i], d1[0]) and torch.equal(p_all[i], p1[0]), (i, r)
    for r in iso:
        i = roots.index(r)
        want_d = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
        want_d[r] = 0
        want_p = want_d.clone()
        want_p[r] = r
        assert torch.equal(d_all[i], want_d) and torch.equal(p_all[i], want_p), r
    h.free()


@pytest.mark.parametrize("n,p", [(1000, 0.012), (777, 0.004), (65, 0.2)])
@pytest.mark.parametrize("kw", [dict(), dict(ids="local", offsets="succinct", relabel=True),
                                dict(layout="plain", relabel=True)])
def test_ragged_vertex_counts(lgmod, n, p, kw):
    """Vertex counts that end inside a 64-vertex word (the multi-source sweeps'
    last word is partial), sparse enough to leave some vertices unreached:
    16 and 40 roots against one-root calls, and oracle rows."""
    g = gg.random_graph(n, p, seed=n, device="cuda")
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    off, col = g.numpy()
    for count in (16, 40):
        roots = gg.pick_roots(g, count, seed=3)
        roots = (roots * ((count + len(roots) - 1) // len(roots)))[:count]  # repeats when few vertices have edges
        d_all, p_all = lgmod.bfs(h, roots)
        for i, r in enumerate(roots):
            d1, p1 = lgmod.bfs(h, [r])
            assert torch.equal(d_all[i], d1[0]) and torch.equal(p_all[i], p1[0]), (count, i, r)
        for i in (0, count - 1):
            d0, p0 = orc.bfs(off.astype(np.uint64), col.view(np.uint32), roots[i],
                             relabeled=bool(kw.get("relabel")))
            np.testing.assert_array_equal(d_all[i].cpu().numpy(), d0)
            np.testing.assert_array_equal(p_all[i].cpu().numpy(), p0)
    h.free()


@pytest.mark.parametrize("counts", [(40, 40), (9, 40)])
def test_multi_root_calls_from_two_threads(lgmod, counts):
    """Two threads, each with its own stream, run multi-root calls on two
    graphs at once: 40 roots (multi-source batches sharing the device's masks
    and lane 0's workspace) or 9 (the lanes): every result equals the same
    call made alone."""
    import threading
    graphs = [gg.kronecker(13, 16, seed=11, device="cuda"), gg.erdos_renyi(13, 8, seed=12, device="cuda")]
    hs = [lgmod.encode(g.row_offsets, g.col, g.n) for g in graphs]
    roots = [gg.pick_roots(g, c, seed=5) for g, c in zip(graphs, counts)]
    ref = [lgmod.bfs(h, r) for h, r in zip(hs, roots)]
    torch.cuda.synchronize()
    out = [[None] * 6, [None] * 6]
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            for k in range(6):
                with torch.cuda.stream(s):
                    d, p = lgmod.bfs(hs[i], roots[i], stream=s)
                s.synchronize()
                out[i][k] = (d, p)
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i in range(2):
        for d, p in out[i]:
            assert torch.equal(d, ref[i][0]) and torch.equal(p, ref[i][1]), i
    for h in hs:
        h.free()


@pytest.mark.parametrize("kw", [dict(), dict(ids="local", offsets="succinct", relabel=True),
                                dict(layout="plain", relabel=True)])
@pytest.mark.parametrize("max_depth", [-1, 3])
def test_many_roots_depths_only(lgmod, kw, max_depth):
    """40 roots without parent rows (the multi-source kernels' depth-only
    forms): depths equal the one-root calls' and the oracle's."""
    g = small_graph("kron13")
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    roots = gg.pick_roots(g, 40, seed=8)
    d_all, p_all = lgmod.bfs(h, roots, parent=False, max_depth=max_depth)
    assert p_all is None
    for i, r in enumerate(roots):
        d1, _ = lgmod.bfs(h, [r], max_depth=max_depth)
        assert torch.equal(d_all[i], d1[0]), (i, r)
    off, col = g.numpy()
    for i in (0, 39):
        d0, _ = orc.bfs(off.astype(np.uint64), col.view(np.uint32), roots[i], max_depth=max_depth,
                        relabeled=bool(kw.get("relabel")))
        np.testing.assert_array_equal(d_all[i].cpu().numpy(), d0)
    h.free()


@pytest.mark.parametrize("kw", [dict(ids="global", offsets="plain-bv"), dict(ids="local", offsets="packed"),
                                dict(ids="local", offsets="plain-bv", relabel=True),
                                dict(ids="local-gap", offsets="packed"),
                                dict(ids="varint-diff", offsets="succinct", relabel=True)],
                         ids=lambda k: "-".join(str(v) for v in k.values()))
def test_many_roots_every_encoding(lgmod, kw):
    """20 roots over the other encodings: bvPL and local packed offsets run
    the multi-source batch, gap and Varint lists (read in order only) run on
    the lanes; every row equals the one-root call."""
    g = small_graph("kron13")
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    roots = gg.pick_roots(g, 20, seed=9)
    d_all, p_all = lgmod.bfs(h, roots)
    for i, r in enumerate(roots):
        d1, p1 = lgmod.bfs(h, [r])
        assert torch.equal(d_all[i], d1[0]) and torch.equal(p_all[i], p1[0]), (i, r)
    h.free()


def test_many_roots_rejected_on_interleaved_offsets(lgmod):
    """bvIL offsets serve the neighbor decode only: a multi-root BFS call is
    rejected as a one-root call is."""
    from paper_2010_15879_amd.lg import LGError, LG_ERR_UNSUPPORTED
    g = small_graph("kron13")
    h = lgmod.encode(g.row_offsets, g.col, g.n, ids="global", offsets="interleaved-bv")
    for count in (1, 20):
        with pytest.raises(LGError) as ei:
            lgmod.bfs(h, gg.pick_roots(g, count, seed=9))
        assert ei.value.status == LG_ERR_UNSUPPORTED, count
    h.free()
