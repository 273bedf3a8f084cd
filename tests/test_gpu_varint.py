"""Varint lists on the GPU (subsection "Incorporating Degree-Minimizing
(DM)": DMf = full labels, DMd = first label and differences, each a
base-128 Varint): every array bit-exact against the oracle, lists decoded
against the input, and BFS and PageRank over them against the oracle."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg
from test_gpu_parity import GRAPHS, PR_L1

pytestmark = pytest.mark.gpu

VARINT = [dict(layout="packed", ids=ids, offsets=offs, relabel=rl)
          for ids in ("varint-full", "varint-diff") for offs in ("packed", "succinct") for rl in (False, True)]


def vid(e):
    return f"{e['ids']}-{e['offsets']}-{'rl' if e['relabel'] else 'id'}"


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


def encode(lgmod, g, e):
    d = g.to("cuda")
    return lgmod.encode(d.row_offsets, d.col, g.n, **e)


def oracle_encoding(g, e):
    off, col = g.numpy()
    return orc.Encoding(off, col, e["ids"], "ef" if e["offsets"] == "succinct" else "packed", e["relabel"])


def check_arrays(h, o, e):
    info = h.info()
    assert info["adj_bits"] == o.U
    np.testing.assert_array_equal(h.export("adj"), o.A)
    if o.ef is None:
        np.testing.assert_array_equal(h.export("offsets"), o.O)
    else:
        np.testing.assert_array_equal(h.export("ef_low"), o.ef.low)
        np.testing.assert_array_equal(h.export("ef_high"), o.ef.high)
        np.testing.assert_array_equal(h.export("ef_select"), o.ef.sel)
    if e["relabel"]:
        np.testing.assert_array_equal(h.export("perm"), o.perm)


@pytest.mark.parametrize("e", VARINT, ids=vid)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_varint_encoding_bit_exact(lgmod, name, e):
    g = GRAPHS[name]
    print(f"[varint encode] {name} {vid(e)}", flush=True)
    h = encode(lgmod, g, e)
    check_arrays(h, oracle_encoding(g, e), e)
    h.free()


def check_decode(lgmod, h, g, e, vs):
    off, col = g.numpy()
    vt = torch.from_numpy(vs).cuda()
    for flags in ["sorted", "original"]:
        o_off, o_ids = lgmod.decode_neighbors(h, vt, flags)
        o_off, o_ids = o_off.cpu().numpy(), o_ids.cpu().numpy()
        for i, v in enumerate(vs):
            got = o_ids[o_off[i]:o_off[i + 1]]
            np.testing.assert_array_equal(np.sort(got) if flags == "original" else got, col[off[v]:off[v + 1]])
    if e["relabel"]:
        perm, inv = orc.dm_permutation(off)
        r_off, r_ids = lgmod.decode_neighbors(h, vt, "raw")
        r_off, r_ids = r_off.cpu().numpy(), r_ids.cpu().numpy()
        for i, x in enumerate(vs):
            np.testing.assert_array_equal(r_ids[r_off[i]:r_off[i + 1]], orc.relabel_row(off, col, perm, inv, int(x)))


@pytest.mark.parametrize("e", VARINT, ids=vid)
@pytest.mark.parametrize("name", ["megastar", "offhub", "kron12", "er12", "star33", "single", "isolated7",
                                  "bigstar", "rand129", "hubtail"])
def test_varint_decode(lgmod, name, e):
    """Lists of many 64-byte steps (the hubs), values of 1 to 3 bytes."""
    g = GRAPHS[name]
    print(f"[varint decode] {name} {vid(e)}", flush=True)
    h = encode(lgmod, g, e)
    rng = np.random.default_rng(12)
    vs = np.unique(np.concatenate([rng.integers(0, g.n, size=min(g.n, 300)), [0, 1, g.n - 1]])).astype(np.int32)
    check_decode(lgmod, h, g, e, vs[vs < g.n])
    h.free()


@pytest.mark.parametrize("e", VARINT, ids=vid)
def test_varint_four_byte_values(lgmod, e):
    """Labels above 2^21 take four bytes; a hub's list mixes one- to four-byte
    differences, and values cross the 64-byte steps at every alignment."""
    n = (1 << 21) + 300
    rng = np.random.default_rng(5)
    far = np.unique(rng.integers(1 << 21, n, size=200))
    near = np.arange(1, 150)
    edges = [(0, int(x)) for x in np.concatenate([near, far])] + [(5, int(x)) for x in far[:40]]
    g = gg.csr_from_edges(n, edges)
    print(f"[varint 4-byte] {vid(e)}", flush=True)
    h = encode(lgmod, g, e)
    check_arrays(h, oracle_encoding(g, e), e)
    vs = np.concatenate([[0, 5, 1, 2, n - 1], far[:20]]).astype(np.int32)
    check_decode(lgmod, h, g, e, vs)
    h.free()


@pytest.mark.parametrize("mode", ["do", "td", "bu"])
@pytest.mark.parametrize("e", VARINT, ids=vid)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_varint_bfs(lgmod, name, e, mode):
    """BFS over Varint lists (read in order): depths and parents bit-exact
    against the oracle, every direction mode."""
    g = GRAPHS[name]
    off, col = g.numpy()
    roots = gg.pick_roots(g, 3, seed=4) or [0]
    if 0 not in roots:
        roots = roots + [0]
    print(f"[varint bfs] {name} {vid(e)} {mode} roots={roots}", flush=True)
    h = encode(lgmod, g, e)
    depth, parent = lgmod.bfs(h, roots, mode=mode)
    depth, parent = depth.cpu().numpy(), parent.cpu().numpy()
    for i, r in enumerate(roots):
        d0, p0 = orc.bfs(off, col, r, relabeled=bool(e["relabel"]))
        np.testing.assert_array_equal(depth[i], d0)
        np.testing.assert_array_equal(parent[i], p0)
    h.free()


def test_varint_bfs_four_byte_labels(lgmod):
    """Values of up to four bytes, hubs longer than the lane's 64-value limit."""
    n = (1 << 21) + 300
    rng = np.random.default_rng(5)
    far = np.unique(rng.integers(1 << 21, n, size=200))
    edges = [(0, int(x)) for x in np.concatenate([np.arange(1, 150), far])] + [(5, int(x)) for x in far[:40]]
    g = gg.csr_from_edges(n, edges)
    off, col = g.numpy()
    for ids in ("varint-full", "varint-diff"):
        h = encode(lgmod, g, dict(layout="packed", ids=ids, offsets="succinct", relabel=False))
        for mode in ("do", "td", "bu"):
            depth, parent = lgmod.bfs(h, [0, int(far[3])], mode=mode)
            for i, r in enumerate([0, int(far[3])]):
                d0, p0 = orc.bfs(off, col, r)
                np.testing.assert_array_equal(depth[i].cpu().numpy(), d0)
                np.testing.assert_array_equal(parent[i].cpu().numpy(), p0)
        h.free()


@pytest.mark.parametrize("e", VARINT, ids=vid)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_varint_pagerank(lgmod, name, e):
    """PageRank over Varint lists: within the FP32 bound of the FP64 oracle,
    and bit-identical from one call to the next."""
    g = GRAPHS[name]
    off, col = g.numpy()
    print(f"[varint pagerank] {name} {vid(e)}", flush=True)
    h = encode(lgmod, g, e)
    for iters in [0, 1, 20]:
        pr = lgmod.pagerank(h, 0.85, iters).cpu().numpy()
        l1 = np.abs(pr.astype(np.float64) - orc.pagerank(off, col, 0.85, iters)).sum()
        assert l1 <= PR_L1, (iters, l1)
    np.testing.assert_array_equal(pr, lgmod.pagerank(h, 0.85, 20).cpu().numpy())
    h.free()


def test_varint_kronecker16(lgmod):
    """Scale 16 with the degree relabeling: DMd and DMf bit-exact, DMd no
    larger than DMf."""
    g = gg.kronecker(16, 16, seed=1)
    sizes = {}
    for ids in ("varint-full", "varint-diff"):
        e = dict(layout="packed", ids=ids, offsets="succinct", relabel=True)
        h = encode(lgmod, g, e)
        o = oracle_encoding(g, e)
        np.testing.assert_array_equal(h.export("adj"), o.A)
        np.testing.assert_array_equal(h.export("ef_low"), o.ef.low)
        sizes[ids] = h.info()["adj_bits"]
        off, col = g.numpy()
        roots = gg.pick_roots(g, 2, seed=6)
        depth, parent = lgmod.bfs(h, roots)
        for i, r in enumerate(roots):
            d0, p0 = orc.bfs(off, col, r, relabeled=True)
            np.testing.assert_array_equal(depth[i].cpu().numpy(), d0)
            np.testing.assert_array_equal(parent[i].cpu().numpy(), p0)
        h.free()
    assert sizes["varint-diff"] <= sizes["varint-full"]


def test_varint_pagerank_chunked_hub(lgmod):
    """A hub whose list spans many 4 KiB chunks with values of one to four
    bytes: the chunk partial sums against the oracle."""
    n = (1 << 21) + 300
    rng = np.random.default_rng(8)
    far = np.unique(rng.integers(1 << 21, n, size=3000))
    edges = [(0, int(x)) for x in np.concatenate([np.arange(1, 6000), far])] + [(5, int(x)) for x in far[:40]]
    g = gg.csr_from_edges(n, edges)
    off, col = g.numpy()
    for ids in ("varint-full", "varint-diff"):
        h = encode(lgmod, g, dict(layout="packed", ids=ids, offsets="succinct", relabel=False))
        pr = lgmod.pagerank(h, 0.85, 10).cpu().numpy().astype(np.float64)
        assert np.abs(pr - orc.pagerank(off, col, 0.85, 10)).sum() <= PR_L1
        h.free()
