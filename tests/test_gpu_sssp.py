"""Weighted graphs and SSSP on the GPU (subsections "Logarithmization of
Edge Weights" and "Accessing an Edge Weight"; SSSP of section "Considered
Algorithms"): the weighted streams bit-exact against the oracle, and the
delta-stepping distances equal to the oracle's Dijkstra distances."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg
from test_gpu_parity import GRAPHS

pytestmark = pytest.mark.gpu

WENC = [
    dict(layout="plain", ids="global", offsets="packed"),
    dict(layout="packed", ids="global", offsets="packed"),
    dict(layout="packed", ids="global", offsets="succinct"),
    dict(layout="packed", ids="local", offsets="packed"),
    dict(layout="packed", ids="local", offsets="succinct"),
]


def wid(e):
    return "plain" if e["layout"] == "plain" else f"{e['ids']}-{e['offsets']}"


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


def encode(lgmod, g, wt, e):
    d = g.to("cuda")
    return lgmod.encode(d.row_offsets, d.col, g.n, weights=torch.from_numpy(wt.astype(np.int32)).cuda(), **e)


def weights_for(g, max_weight=255, seed=1):
    return gg.edge_weights(g, max_weight, seed=seed).numpy().astype(np.uint32)


@pytest.mark.parametrize("e", WENC, ids=wid)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_weighted_encoding_bit_exact(lgmod, name, e):
    g = GRAPHS[name]
    wt = weights_for(g)
    print(f"[weighted encode] {name} {wid(e)}", flush=True)
    h = encode(lgmod, g, wt, e)
    off, col = g.numpy()
    info = h.info()
    if e["layout"] == "plain":
        np.testing.assert_array_equal(h.export("adj"), col)
        np.testing.assert_array_equal(h.export("weights"), wt)
        assert info["bytes_weights"] >= 4 * col.size
    else:
        o = orc.Encoding(off, col, e["ids"], "ef" if e["offsets"] == "succinct" else "packed", weights=wt)
        assert info["weight_bits"] == o.omega
        assert info["adj_bits"] == o.U
        np.testing.assert_array_equal(h.export("adj"), o.A)
        if o.ef is None:
            np.testing.assert_array_equal(h.export("offsets"), o.O)
        else:
            np.testing.assert_array_equal(h.export("ef_low"), o.ef.low)
            np.testing.assert_array_equal(h.export("ef_high"), o.ef.high)
            np.testing.assert_array_equal(h.export("ef_select"), o.ef.sel)
        if e["ids"] == "local":
            np.testing.assert_array_equal(h.export("widths"), o.W)
    h.free()


def roots_of(g):
    off, _ = g.numpy()
    deg = off[1:] - off[:-1]
    rs = {0, g.n - 1}
    nz = np.nonzero(deg)[0]
    if nz.size:
        rs.add(int(nz[len(nz) // 2]))
        rs.add(int(nz[np.argmax(deg[nz])]))
    return sorted(rs)


@pytest.mark.parametrize("e", WENC, ids=wid)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_sssp_matches_oracle(lgmod, name, e):
    g = GRAPHS[name]
    wt = weights_for(g, 255, seed=3)
    off, col = g.numpy()
    h = encode(lgmod, g, wt, e)
    for root in roots_of(g):
        expect = orc.sssp(off, col, wt, root)
        for delta in (0, 1, 37, 100000):
            print(f"[sssp] {name} {wid(e)} root={root} delta={delta}", flush=True)
            got = lgmod.sssp(h, root, delta).cpu().numpy()
            np.testing.assert_array_equal(got, expect)
    h.free()


@pytest.mark.parametrize("e", WENC[1:], ids=wid)
def test_sssp_wide_and_zero_weights(lgmod, e):
    """Weights of 31 bits (distances beyond 32 bits) and weights of 0."""
    g = GRAPHS["kron12"]
    off, col = g.numpy()
    for wt in (weights_for(g, (1 << 31) - 1, seed=5), weights_for(g, 3, seed=6) - 1):
        h = encode(lgmod, g, wt, e)
        for root in roots_of(g):
            print(f"[sssp wide/zero] {wid(e)} root={root} max={int(wt.max())}", flush=True)
            np.testing.assert_array_equal(lgmod.sssp(h, root).cpu().numpy(), orc.sssp(off, col, wt, root))
        h.free()


def test_sssp_kronecker16(lgmod):
    g = gg.kronecker(16, 16, seed=1)
    off, col = g.numpy()
    wt = weights_for(g, 255, seed=1)
    roots = gg.pick_roots(g, 4, seed=3)
    for e in (WENC[0], WENC[4]):
        h = encode(lgmod, g, wt, e)
        for r in roots:
            print(f"[sssp kron16] {wid(e)} root={r}", flush=True)
            np.testing.assert_array_equal(lgmod.sssp(h, r).cpu().numpy(), orc.sssp(off, col, wt, r))
        h.free()


def test_weighted_unsupported(lgmod):
    from paper_2010_15879_amd.lg import LGError, LG_ERR_UNSUPPORTED
    g = GRAPHS["kron12"]
    wt = weights_for(g)
    h = encode(lgmod, g, wt, WENC[4])
    root = gg.pick_roots(g, 1, seed=1)
    for call in (lambda: lgmod.bfs(h, root), lambda: lgmod.pagerank(h, 0.85, 2),
                 lambda: lgmod.decode_neighbors(h, torch.tensor([0], dtype=torch.int32, device="cuda")),
                 lambda: lgmod.BatchPlan([h], [(0, root[0])])):
        with pytest.raises(LGError) as ei:
            call()
        assert ei.value.status == LG_ERR_UNSUPPORTED
    h.free()
    d = g.to("cuda")
    hu = lgmod.encode(d.row_offsets, d.col, g.n)
    with pytest.raises(LGError) as ei:
        lgmod.sssp(hu, root[0])
    assert ei.value.status == LG_ERR_UNSUPPORTED
    hu.free()
    for bad in (dict(layout="packed", ids="local-gap", offsets="packed"),
                dict(layout="packed", ids="varint-diff", offsets="packed")):
        with pytest.raises(LGError) as ei:
            encode(lgmod, g, wt, bad)
        assert ei.value.status == LG_ERR_UNSUPPORTED


def test_weighted_plain_traversals(lgmod):
    """A weighted plain graph still serves BFS and PageRank."""
    g = GRAPHS["kron12"]
    off, col = g.numpy()
    h = encode(lgmod, g, weights_for(g), WENC[0])
    root = gg.pick_roots(g, 1, seed=2)
    depth, _ = lgmod.bfs(h, root)
    np.testing.assert_array_equal(depth.cpu().numpy().reshape(-1), orc.bfs(off, col, root[0])[0])
    pr = lgmod.pagerank(h, 0.85, 5).cpu().numpy().astype(np.float64)
    assert np.abs(pr - orc.pagerank(off, col, 0.85, 5)).sum() <= 1e-5
    h.free()


def test_sssp_invalid_arguments(lgmod):
    from paper_2010_15879_amd.lg import LGError, LG_ERR_INVALID
    g = GRAPHS["kron12"]
    h = encode(lgmod, g, weights_for(g), WENC[3])
    with pytest.raises(LGError) as ei:
        lgmod.sssp(h, g.n)
    assert ei.value.status == LG_ERR_INVALID
    h.free()
    d = g.to("cuda")
    with pytest.raises(ValueError):
        lgmod.encode(d.row_offsets, d.col, g.n, weights=torch.ones(3, dtype=torch.int32, device="cuda"))


WREL = [
    dict(layout="packed", ids="local", offsets="succinct", relabel=True),
    dict(layout="packed", ids="global", offsets="packed", relabel="greedy"),
    dict(layout="plain", relabel=True),
]


@pytest.mark.parametrize("e", WREL, ids=["local-ef-dm", "global-packed-greedy", "plain-dm"])
@pytest.mark.parametrize("name", ["kron12", "er12", "megastar", "hubtail", "rand129", "isolated7", "bigstar"])
def test_weighted_relabeled(lgmod, name, e):
    """Weights under a relabeling: every entry keeps its edge's weight
    (streams bit-exact against the oracle), and the distances come back by
    original ID, equal to the oracle's Dijkstra on the original graph."""
    g = GRAPHS[name]
    off, col = g.numpy()
    wt = weights_for(g, 255, seed=9)
    print(f"[weighted relabel] {name} {e}", flush=True)
    h = encode(lgmod, g, wt, e)
    o = orc.Encoding(off, col, e.get("ids", "global"), "ef" if e.get("offsets") == "succinct" else "packed",
                     e["relabel"], weights=wt)
    if e["layout"] == "plain":
        np.testing.assert_array_equal(h.export("adj"), o.col)
        np.testing.assert_array_equal(h.export("weights"), o.weights)
    else:
        np.testing.assert_array_equal(h.export("adj"), o.A)
    for root in roots_of(g):
        np.testing.assert_array_equal(lgmod.sssp(h, root).cpu().numpy(), orc.sssp(off, col, wt, root))
    h.free()
