"""PageRank by propagation blocking (unrelabeled graphs of at least 2^22
vertices): the whole score vector within L1 1e-5 of the oracle's FP64
PageRank after 1 and 20 iterations, in every layout the path serves, and bit
for bit the same on a second call (the sums are exact fixed-point sums).
Kronecker scale 22 brings hub lists cut into segments and blocks of
vertices without edges; Erdos-Renyi scale 22 uniform lists."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg

pytestmark = pytest.mark.gpu

LAYOUTS = [dict(ids="global", offsets="packed"), dict(ids="local", offsets="succinct"),
           dict(ids="global", offsets="plain-bv"), dict(ids="local", offsets="packed"), dict(layout="plain")]


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


@pytest.fixture(scope="module", params=["er22", "kron22"])
def graph(request):
    if request.param == "er22":
        g = gg.erdos_renyi(22, 16, seed=4, device="cuda")
    else:
        g = gg.kronecker(22, 16, seed=4, device="cuda")
    off, col = g.numpy()
    off, col = off.astype(np.uint64), col.view(np.uint32)
    print(f"[pb] {request.param}: n={g.n} M={g.m}; oracle", flush=True)
    want = {t: orc.pagerank_par(off, col, 0.85, t) for t in (1, 20)}
    return request.param, g, want


@pytest.mark.parametrize("kw", LAYOUTS, ids=lambda k: "-".join(k.values()))
def test_pagerank_pb_parity(lgmod, graph, kw):
    name, g, want = graph
    assert g.n >= 1 << 22
    print(f"[pb] {name} {kw}", flush=True)
    h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
    for t in (1, 20):
        pr = lgmod.pagerank(h, 0.85, t)
        again = lgmod.pagerank(h, 0.85, t)
        assert torch.equal(pr, again), "scores differ between two calls"
        l1 = float(np.abs(pr.cpu().numpy().astype(np.float64) - want[t]).sum())
        assert l1 <= 1e-5, (t, l1)
    z = lgmod.pagerank(h, 0.85, 0).cpu().numpy()
    np.testing.assert_allclose(z, 1.0 / g.n, rtol=0, atol=0)
    h.free()


@pytest.mark.parametrize("edges", ["none", "sparse"])
def test_pagerank_pb_nearly_empty(lgmod, edges):
    """2^22 vertices with no edges, or a few thousand edges and one hub: most
    level-1 workgroups get no entries (or none at all), and the scores still
    match the oracle."""
    n = 1 << 22
    if edges == "none":
        g = gg.csr_from_edges(n, [], device="cuda")
    else:
        rng = np.random.default_rng(5)
        src = rng.integers(0, n, 3000)
        dst = rng.integers(0, n, 3000)
        hub = np.full(2000, 12345)
        leaves = rng.integers(0, n, 2000)
        s = torch.from_numpy(np.concatenate([src, hub])).cuda()
        d = torch.from_numpy(np.concatenate([dst, leaves])).cuda()
        g = gg.canonical_csr(n, s, d)
    off, col = g.numpy()
    off, col = off.astype(np.uint64), col.view(np.uint32)
    for kw in (dict(ids="global", offsets="packed"), dict(layout="plain")):
        print(f"[pb] nearly empty ({edges}, m={g.m}) {kw}", flush=True)
        h = lgmod.encode(g.row_offsets, g.col, g.n, **kw)
        for t in (1, 20):
            pr = lgmod.pagerank(h, 0.85, t).cpu().numpy().astype(np.float64)
            l1 = float(np.abs(pr - orc.pagerank_par(off, col, 0.85, t)).sum())
            assert l1 <= 1e-5, (edges, kw, t, l1)
        h.free()
