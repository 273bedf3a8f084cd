"""GPU parity: every array of the encoding, every decoded list and every
BFS depth/parent is bit-exact against the CPU oracle; FP32 PageRank is
within L1 <= 1e-5 of the FP64 oracle (and sums to 1 within 1e-5).

Graphs: adversarial tiny cases, several tiles with a ragged tail, and the
Kronecker scale-16 configuration."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg

pytestmark = pytest.mark.gpu

PR_L1 = 1e-5

ENCODINGS = [
    dict(layout="packed", ids="global", offsets="packed", relabel=False),
    dict(layout="packed", ids="global", offsets="succinct", relabel=False),
    dict(layout="packed", ids="local", offsets="packed", relabel=False),
    dict(layout="packed", ids="local", offsets="succinct", relabel=True),
    dict(layout="packed", ids="global", offsets="packed", relabel=True),
    dict(layout="packed", ids="local", offsets="succinct", relabel=False),
    dict(layout="plain", relabel=False),
    dict(layout="plain", relabel=True),
    dict(layout="packed", ids="local", offsets="succinct", relabel="greedy"),
    dict(layout="plain", relabel="greedy"),
]


def oracle_perm(off, col, relabel):
    """(perm, inv) of the oracle for the encoding's relabeling."""
    return orc.greedy_permutation(off, col) if relabel == "greedy" else orc.dm_permutation(off)


def oracle_bfs(off, col, root, relabel, max_depth=-1):
    """Depths and parents (smallest stored label among the candidates)."""
    if relabel == "greedy":
        return orc.bfs(off, col, root, max_depth=max_depth, labels=oracle_perm(off, col, relabel)[1])
    return orc.bfs(off, col, root, max_depth=max_depth, relabeled=bool(relabel))


def enc_id(e):
    return "-".join(str(v) if not isinstance(v, bool) else ("rl" if v else "id") for v in e.values())


def _tiny_graphs():
    G = {}
    G["single"] = gg.csr_from_edges(1, [])
    G["edge"] = gg.csr_from_edges(2, [(0, 1)])
    G["isolated7"] = gg.csr_from_edges(7, [])
    G["path9"] = gg.csr_from_edges(9, [(i, i + 1) for i in range(8)])
    G["star33"] = gg.csr_from_edges(33, [(0, i) for i in range(1, 33)])
    G["clique12"] = gg.csr_from_edges(12, [(i, j) for i in range(12) for j in range(i + 1, 12)])
    G["only0"] = gg.csr_from_edges(5, [(0, 4), (1, 2)])
    G["hubtail"] = gg.csr_from_edges(70, [(69, i) for i in range(69)] + [(3, 4)])
    # degrees 64 and 65 straddle the heavy-vertex threshold of the traversal kernels
    G["deg64_65"] = gg.csr_from_edges(200, [(0, i) for i in range(2, 66)] + [(1, i) for i in range(100, 165)]
                                      + [(2, 100)])
    # a hub of degree 3000: below the PageRank split, so one unit walks its
    # whole list 64 entries at a time
    G["bigstar"] = gg.csr_from_edges(3001, [(0, i) for i in range(1, 3001)] + [(5, 6), (6, 7)])
    # a hub so large that its gap in the Elias-Fano upper bits spans more than
    # 64 words (the per-lane select fallback of the sweep kernels)
    G["megastar"] = gg.csr_from_edges(20001, [(0, i) for i in range(1, 20001)] + [(7, 8), (8, 9)])
    # the hub is row 1, not row 0: the 8,192-entry pieces of its 64-row block
    # start in the middle of a 64-bit word, so neighbouring pieces share the
    # packed words at their boundaries
    G["offhub"] = gg.csr_from_edges(20002, [(0, 2)] + [(1, i) for i in range(2, 20002)])
    for n in [63, 64, 65, 127, 129]:
        G[f"rand{n}"] = gg.random_graph(n, 0.07, seed=n)
    G["kron12"] = gg.kronecker(12, 16, seed=1)
    G["er12"] = gg.erdos_renyi(12, 16, seed=2)
    G["kron10ef4"] = gg.kronecker(10, 4, seed=7)
    return G


GRAPHS = _tiny_graphs()


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    assert torch.cuda.is_available()
    return lg


def oracle_encoding(g, e):
    off, col = g.numpy()
    if e["layout"] == "plain":
        return None
    return orc.Encoding(off, col, e["ids"], "ef" if e["offsets"] == "succinct" else "packed", e["relabel"])


def encode(lgmod, g, e):
    d = g.to("cuda")
    kw = {k: v for k, v in e.items()}
    return lgmod.encode(d.row_offsets, d.col, g.n, **kw)


@pytest.mark.parametrize("e", ENCODINGS, ids=enc_id)
@pytest.mark.parametrize("name", list(GRAPHS))
def test_encoding_bit_exact(lgmod, name, e):
    g = GRAPHS[name]
    print(f"[encode] {name} n={g.n} m={g.m} {e}", flush=True)
    h = encode(lgmod, g, e)
    off, col = g.numpy()
    if e["layout"] == "plain":
        if e["relabel"]:
            perm, inv = oracle_perm(off, col, e["relabel"])
            off, col = orc.relabel(off, col, perm, inv)
            np.testing.assert_array_equal(h.export("perm"), perm)
            np.testing.assert_array_equal(h.export("inv"), inv)
        np.testing.assert_array_equal(h.export("adj"), col)
        np.testing.assert_array_equal(h.export("offsets").astype(np.uint64), off)
        h.free()
        return
    o = oracle_encoding(g, e)
    info = h.info()
    assert info["adj_bits"] == o.U
    assert info["s"] == o.s
    np.testing.assert_array_equal(h.export("adj"), o.A)
    if o.ef is None:
        assert info["w_offset"] == o.wO
        np.testing.assert_array_equal(h.export("offsets"), o.O)
    else:
        assert info["ef_l"] == o.ef.l and info["ef_high_bits"] == o.ef.hbits
        np.testing.assert_array_equal(h.export("ef_low"), o.ef.low)
        np.testing.assert_array_equal(h.export("ef_high"), o.ef.high)
        np.testing.assert_array_equal(h.export("ef_rank"), o.ef.rank_sb)
        np.testing.assert_array_equal(h.export("ef_select"), o.ef.sel)
    if e["ids"] == "local":
        assert info["F"] == o.F
        np.testing.assert_array_equal(h.export("widths"), o.W)
    if e["relabel"]:
        np.testing.assert_array_equal(h.export("perm"), o.perm)
        np.testing.assert_array_equal(h.export("inv"), o.inv)
    h.free()


@pytest.mark.parametrize("e", ENCODINGS, ids=enc_id)
@pytest.mark.parametrize("name", ["star33", "hubtail", "rand65", "kron12", "er12", "single", "isolated7",
                                  "bigstar"])
def test_decode_neighbors(lgmod, name, e):
    g = GRAPHS[name]
    print(f"[decode] {name} {e}", flush=True)
    h = encode(lgmod, g, e)
    off, col = g.numpy()
    rng = np.random.default_rng(5)
    vs = np.unique(np.concatenate([rng.integers(0, g.n, size=min(g.n, 300)), [0, g.n - 1]])).astype(np.int32)
    vt = torch.from_numpy(vs).cuda()
    o_off, o_ids = lgmod.decode_neighbors(h, vt, "sorted")
    o_off, o_ids = o_off.cpu().numpy(), o_ids.cpu().numpy()
    for i, v in enumerate(vs):
        np.testing.assert_array_equal(o_ids[o_off[i]:o_off[i + 1]], col[off[v]:off[v + 1]])
    # stored order / stored labels
    if e["relabel"]:
        perm, inv = oracle_perm(off, col, e["relabel"])
        r_off, r_ids = lgmod.decode_neighbors(h, vt, "raw")
        r_off, r_ids = r_off.cpu().numpy(), r_ids.cpu().numpy()
        for i, x in enumerate(vs):
            np.testing.assert_array_equal(r_ids[r_off[i]:r_off[i + 1]], orc.relabel_row(off, col, perm, inv, int(x)))
        s_off, s_ids = lgmod.decode_neighbors(h, vt, "original")
        s_off, s_ids = s_off.cpu().numpy(), s_ids.cpu().numpy()
        for i, v in enumerate(vs):
            np.testing.assert_array_equal(np.sort(s_ids[s_off[i]:s_off[i + 1]]), col[off[v]:off[v + 1]])
    h.free()


@pytest.mark.parametrize("mode", ["do", "td", "bu"])
@pytest.mark.parametrize("e", ENCODINGS, ids=enc_id)
@pytest.mark.parametrize("name", ["path9", "star33", "clique12", "only0", "hubtail", "rand64", "rand129",
                                  "kron12", "er12", "kron10ef4", "single", "edge", "deg64_65", "bigstar",
                                  "megastar"])
def test_bfs_bit_exact(lgmod, name, e, mode):
    g = GRAPHS[name]
    off, col = g.numpy()
    roots = gg.pick_roots(g, 3, seed=4) or [0]
    if 0 not in roots:
        roots = roots + [0]  # vertex 0 may be isolated: a valid BFS too
    print(f"[bfs] {name} {e} {mode} roots={roots}", flush=True)
    h = encode(lgmod, g, e)
    depth, parent = lgmod.bfs(h, roots, mode=mode)
    depth, parent = depth.cpu().numpy(), parent.cpu().numpy()
    for i, r in enumerate(roots):
        d0, p0 = oracle_bfs(off, col, r, e["relabel"])
        np.testing.assert_array_equal(depth[i], d0)
        np.testing.assert_array_equal(parent[i], p0)
    h.free()


@pytest.mark.parametrize("e", ENCODINGS[:4] + ENCODINGS[6:], ids=enc_id)
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_bfs_k_hop(lgmod, e, k):
    g = GRAPHS["kron12"]
    off, col = g.numpy()
    roots = gg.pick_roots(g, 4, seed=9)
    print(f"[khop] k={k} {e}", flush=True)
    h = encode(lgmod, g, e)
    depth, parent = lgmod.bfs(h, roots, max_depth=k)
    for i, r in enumerate(roots):
        d0, p0 = oracle_bfs(off, col, r, e["relabel"], max_depth=k)
        np.testing.assert_array_equal(depth[i].cpu().numpy(), d0)
        np.testing.assert_array_equal(parent[i].cpu().numpy(), p0)
    h.free()


def test_bfs_without_parents(lgmod):
    g = GRAPHS["kron12"]
    off, col = g.numpy()
    roots = gg.pick_roots(g, 2, seed=3)
    for e in [ENCODINGS[0], ENCODINGS[3]]:
        h = encode(lgmod, g, e)
        depth, par = lgmod.bfs(h, roots, parent=False)
        assert par is None
        for i, r in enumerate(roots):
            d0, _ = orc.bfs(off, col, r)
            np.testing.assert_array_equal(depth[i].cpu().numpy(), d0)
        h.free()


@pytest.mark.parametrize("e", ENCODINGS, ids=enc_id)
@pytest.mark.parametrize("name", ["star33", "clique12", "isolated7", "single", "hubtail", "rand127", "kron12",
                                  "er12", "deg64_65", "bigstar", "megastar"])
def test_pagerank_l1(lgmod, name, e):
    g = GRAPHS[name]
    off, col = g.numpy()
    print(f"[pagerank] {name} {e}", flush=True)
    h = encode(lgmod, g, e)
    for iters in [0, 1, 20]:
        pr = lgmod.pagerank(h, 0.85, iters).cpu().numpy().astype(np.float64)
        pr64 = orc.pagerank(off, col, 0.85, iters)
        l1 = np.abs(pr - pr64).sum()
        assert l1 <= PR_L1, (iters, l1)
        assert abs(pr.sum() - 1.0) <= PR_L1
    h.free()


def test_pagerank_reproducible(lgmod):
    g = GRAPHS["kron12"]
    h = encode(lgmod, g, ENCODINGS[3])
    a = lgmod.pagerank(h, 0.85, 20).cpu().numpy()
    b = lgmod.pagerank(h, 0.85, 20).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    h.free()


def test_invalid_inputs_rejected(lgmod):
    from paper_2010_15879_amd.lg import LGError, LG_ERR_INVALID
    cases = {
        "unsorted": (np.array([0, 2, 3, 4], np.int64), np.array([2, 1, 0, 0], np.int32)),
        "asymmetric": (np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32)),
        "self_loop": (np.array([0, 1, 1], np.int64), np.array([0], np.int32)),
        "id_out_of_range": (np.array([0, 1, 2], np.int64), np.array([5, 0], np.int32)),
        "bad_offsets": (np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32)),
    }
    for name, (off, col) in cases.items():
        print(f"[invalid] {name}", flush=True)
        with pytest.raises(LGError) as ei:
            lgmod.encode(torch.from_numpy(off).cuda(), torch.from_numpy(col).cuda(), off.size - 1)
        assert ei.value.status == LG_ERR_INVALID, name
    g = GRAPHS["path9"]
    h = encode(lgmod, g, ENCODINGS[0])
    with pytest.raises(LGError):
        lgmod.bfs(h, [g.n])
    with pytest.raises(LGError):
        lgmod.decode_neighbors(h, torch.tensor([g.n], dtype=torch.int32, device="cuda"))
    h.free()


def _rewired(g):
    """g with two entries retargeted so that every in-degree equals the
    out-degree but the graph is not symmetric: a->b, c->d become a->d, c->b
    (b->a and d->c stay)."""
    off, col = g.numpy()
    off = off.astype(np.int64)
    rows = [list(col[off[v]:off[v + 1]]) for v in range(g.n)]
    rng = np.random.default_rng(11)
    while True:
        a, c = (int(x) for x in rng.integers(g.n, size=2))
        if a == c or not rows[a] or not rows[c]:
            continue
        b, d = int(rows[a][rng.integers(len(rows[a]))]), int(rows[c][rng.integers(len(rows[c]))])
        if len({a, b, c, d}) < 4 or d in rows[a] or b in rows[c]:
            continue
        break
    rows[a] = sorted(set(rows[a]) - {b} | {d})
    rows[c] = sorted(set(rows[c]) - {d} | {b})
    noff = np.zeros(g.n + 1, np.int64)
    noff[1:] = np.cumsum([len(r) for r in rows])
    return noff, np.concatenate([np.array(r, np.int32) for r in rows])


@pytest.mark.parametrize("layout", ["packed", "plain"])
def test_invalid_inputs_rejected_relabel(lgmod, layout):
    """Invalid graphs are rejected with the degree relabeling too, including
    graphs whose in-degrees equal their out-degrees but that are not
    symmetric (a directed 3-cycle, two retargeted entries)."""
    from paper_2010_15879_amd.lg import LGError, LG_ERR_INVALID
    cases = {
        "unsorted": (np.array([0, 2, 3, 4], np.int64), np.array([2, 1, 0, 0], np.int32)),
        "asymmetric": (np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32)),
        "cycle3": (np.array([0, 1, 2, 3], np.int64), np.array([1, 2, 0], np.int32)),
        "self_loop": (np.array([0, 1, 1], np.int64), np.array([0], np.int32)),
        "rewired_kron10": _rewired(gg.kronecker(10, 8, seed=4)),
        "rewired_er9": _rewired(gg.erdos_renyi(9, 6, seed=2)),
    }
    for name, (off, col) in cases.items():
        print(f"[invalid relabel {layout}] {name}", flush=True)
        with pytest.raises(LGError) as ei:
            lgmod.encode(torch.from_numpy(off).cuda(), torch.from_numpy(col).cuda(), off.size - 1,
                         layout=layout, relabel=True)
        assert ei.value.status == LG_ERR_INVALID, name
        assert "not-symmetric" in str(ei.value) or name in ("unsorted", "self_loop"), name
    # the same graphs before rewiring are accepted
    for g in [gg.kronecker(10, 8, seed=4), gg.erdos_renyi(9, 6, seed=2)]:
        h = encode(lgmod, g, dict(layout=layout, relabel=True) if layout == "plain" else ENCODINGS[3])
        h.free()


def test_decode_capacity_error(lgmod):
    from paper_2010_15879_amd.lg import LGError, LG_ERR_CAPACITY
    g = GRAPHS["star33"]
    h = encode(lgmod, g, ENCODINGS[0])
    vt = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    with pytest.raises(LGError) as ei:
        lgmod.decode_neighbors(h, vt, cap=10)
    assert ei.value.status == LG_ERR_CAPACITY
    h.free()


@pytest.mark.parametrize("e", [ENCODINGS[0], ENCODINGS[3], ENCODINGS[6], ENCODINGS[7], ENCODINGS[8]], ids=enc_id)
def test_kronecker16_config(lgmod, e):
    """Kronecker scale 16, edge factor 16, seed 1: 64 roots, 20 PR iterations."""
    g = gg.kronecker(16, 16, seed=1)
    off, col = g.numpy()
    print(f"[kron16] n={g.n} m={g.m} {e}", flush=True)
    h = encode(lgmod, g, e)
    if e["layout"] == "packed":
        o = oracle_encoding(g, e)
        np.testing.assert_array_equal(h.export("adj"), o.A)
    roots = gg.pick_roots(g, 64, seed=1)
    depth, parent = lgmod.bfs(h, roots)
    depth, parent = depth.cpu().numpy(), parent.cpu().numpy()
    for i, r in enumerate(roots):  # every one of the 64 roots
        d0, p0 = oracle_bfs(off, col, r, e["relabel"])
        np.testing.assert_array_equal(depth[i], d0)
        np.testing.assert_array_equal(parent[i], p0)
    pr = lgmod.pagerank(h, 0.85, 20).cpu().numpy().astype(np.float64)
    pr64 = orc.pagerank(off, col, 0.85, 20)
    assert np.abs(pr - pr64).sum() <= PR_L1
    h.free()
