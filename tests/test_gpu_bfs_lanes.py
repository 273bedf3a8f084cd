"""lg_bfs with many roots runs them a few at a time on internal streams:
every row must equal the result of a call with that root alone, and work on
the caller's stream must be ordered around the call."""

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


@pytest.mark.parametrize("kw", [dict(), dict(ids="local", offsets="succinct", relabel=True),
                                dict(layout="plain", relabel=True)])
@pytest.mark.parametrize("max_depth", [-1, 2])
def test_many_roots_equal_one_at_a_time(lgmod, kw, max_depth):
    g = gg.kronecker(13, 16, seed=5, device="cuda")
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    roots = gg.pick_roots(g, 37, seed=2)
    d_all, p_all = lgmod.bfs(h, roots, max_depth=max_depth)
    for i, r in enumerate(roots):
        d1, p1 = lgmod.bfs(h, [r], max_depth=max_depth)
        assert torch.equal(d_all[i], d1[0]) and torch.equal(p_all[i], p1[0]), (i, r)
    off, col = g.numpy()
    for i in [0, 17, len(roots) - 1]:
        d0, p0 = orc.bfs(off.astype(np.uint64), col.view(np.uint32), roots[i], max_depth=max_depth,
                         relabeled=bool(kw.get("relabel")))
        np.testing.assert_array_equal(d_all[i].cpu().numpy(), d0)
        np.testing.assert_array_equal(p_all[i].cpu().numpy(), p0)
    h.free()


def test_stream_order_around_the_call(lgmod):
    """Outputs written on the caller's stream before the call are overwritten by
    it, and a kernel queued after the call sees the final rows."""
    g = gg.kronecker(12, 16, seed=9, device="cuda")
    h = lgmod.encode(g.row_offsets, g.col, g.n)
    roots = gg.pick_roots(g, 9, seed=3)
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
