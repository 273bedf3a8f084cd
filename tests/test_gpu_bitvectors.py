"""GPU parity of the plain (bvPL) and interleaved (bvIL) bit-vector offsets
(subsection "Arrays of Offsets vs. Bit Vectors for O"): every array bit-exact
against the oracle, every decoded list (both neighbor-decode entry points)
equal to the input, and for bvPL -- which every operation reads -- BFS trees
and PageRank against the oracle; bvIL graphs refuse the other operations."""

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2010_15879_amd import graphgen as gg
from test_gpu_parity import GRAPHS

pytestmark = pytest.mark.gpu

VARIANTS = [
    ("plain-bv", "global", False), ("plain-bv", "local", False), ("plain-bv", "local", True),
    ("interleaved-bv", "global", False), ("interleaved-bv", "local", False), ("interleaved-bv", "local", True),
]
NAMES = ["single", "edge", "isolated7", "path9", "star33", "only0", "deg64_65", "bigstar", "megastar", "offhub",
         "rand65", "rand129", "kron12", "er12"]


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


def vid(v):
    return "-".join(str(x) for x in v)


def check_arrays(h, o, mode):
    info = h.info()
    assert info["adj_bits"] == o.U
    np.testing.assert_array_equal(h.export("adj"), o.A)
    if mode == "plain-bv":
        assert info["ef_l"] == 0 and info["ef_high_bits"] == o.bv.nbits
        np.testing.assert_array_equal(h.export("ef_high"), o.bv.bits)
        np.testing.assert_array_equal(h.export("ef_rank"), o.bv.rank_sb)
        np.testing.assert_array_equal(h.export("ef_select"), o.bv.sel)
        assert info["bytes_offsets"] == o.bv.bits.size * 8 + o.bv.rank_sb.size * 4 + o.bv.sel.size * 4
    else:
        assert info["ef_high_bits"] == o.bvil.nbits
        np.testing.assert_array_equal(h.export("bv_interleaved"), o.bvil.words)
        assert info["bytes_offsets"] == o.bvil.words.size * 8


def check_decode(lgmod, h, g, off, col, o):
    vt = torch.arange(g.n, dtype=torch.int32, device="cuda")
    d_off, d_ids = lgmod.decode_neighbors(h, vt, "sorted")
    np.testing.assert_array_equal(d_off.cpu().numpy().astype(np.uint64), off)
    np.testing.assert_array_equal(d_ids.cpu().numpy(), col)
    r_off, r_ids = lgmod.decode_neighbors(h, vt, "raw")
    raw_ids = r_ids.cpu().numpy()
    r_off = r_off.cpu().numpy()
    for x in range(0, g.n, max(1, g.n // 200)):
        np.testing.assert_array_equal(raw_ids[r_off[x]:r_off[x + 1]], o.neighbors(x))
    # the allocation-free decode of the first vertices in stored order
    k = min(g.n, 4096)
    vk = vt[:k].contiguous()
    off2 = torch.empty(k + 1, dtype=torch.int64, device="cuda")
    ids2 = torch.empty(max(int(d_off[k].item()), 1), dtype=torch.int32, device="cuda")
    assert lgmod.decode_neighbors_noalloc(h, vk, off2, ids2, "sorted") == lgmod.LG_OK
    np.testing.assert_array_equal(off2.cpu().numpy(), d_off[:k + 1].cpu().numpy())
    np.testing.assert_array_equal(ids2[:int(off2[-1].item())].cpu().numpy(), col[:int(off[k])])


@pytest.mark.parametrize("v", VARIANTS, ids=vid)
@pytest.mark.parametrize("name", NAMES)
def test_bit_vector_offsets(lgmod, name, v):
    mode, ids, rl = v
    g = GRAPHS[name]
    print(f"[bitvec] {name} n={g.n} m={g.m} {v}", flush=True)
    off, col = g.numpy()
    off, col = off.astype(np.uint64), col.view(np.uint32)
    d = g.to("cuda")
    h = lgmod.encode(d.row_offsets, d.col, g.n, ids=ids, offsets=mode, relabel=rl)
    o = orc.Encoding(off, col, ids, mode, rl)
    check_arrays(h, o, mode)
    check_decode(lgmod, h, g, off, col, o)
    roots = gg.pick_roots(g, 2, seed=3) or [0]
    if mode == "plain-bv":
        depth, parent = lgmod.bfs(h, roots)
        for i, r in enumerate(roots):
            d0, p0 = orc.bfs(off, col, r, relabeled=rl)
            np.testing.assert_array_equal(depth[i].cpu().numpy(), d0)
            np.testing.assert_array_equal(parent[i].cpu().numpy(), p0)
        pr = lgmod.pagerank(h, 0.85, 20).cpu().numpy().astype(np.float64)
        assert np.abs(pr - orc.pagerank(off, col, 0.85, 20)).sum() <= 1e-5
    else:
        for call in (lambda: lgmod.bfs(h, roots[:1]), lambda: lgmod.pagerank(h, 0.85, 2)):
            with pytest.raises(lgmod.LGError) as ex:
                call()
            assert ex.value.status == lgmod.LG_ERR_UNSUPPORTED
    h.free()


@pytest.mark.parametrize("mode", ["plain-bv", "interleaved-bv"])
def test_kronecker16(lgmod, mode):
    g = gg.kronecker(16, 16, seed=1)
    off, col = g.numpy()
    off, col = off.astype(np.uint64), col.view(np.uint32)
    d = g.to("cuda")
    for ids in ("global", "local"):
        print(f"[bitvec] kronecker s16 {mode} {ids}", flush=True)
        h = lgmod.encode(d.row_offsets, d.col, g.n, ids=ids, offsets=mode)
        o = orc.Encoding(off, col, ids, mode, False)
        check_arrays(h, o, mode)
        check_decode(lgmod, h, g, off, col, o)
        h.free()


def test_unsupported_combinations(lgmod):
    g = GRAPHS["kron12"].to("cuda")
    for ids in ("local-gap", "varint-diff"):
        with pytest.raises(lgmod.LGError) as ex:
            lgmod.encode(g.row_offsets, g.col, g.n, ids=ids, offsets="interleaved-bv")
        assert ex.value.status == lgmod.LG_ERR_UNSUPPORTED
    w = torch.ones(g.m, dtype=torch.int32, device="cuda")
    with pytest.raises(lgmod.LGError) as ex:
        lgmod.encode(g.row_offsets, g.col, g.n, offsets="interleaved-bv", weights=w)
    assert ex.value.status == lgmod.LG_ERR_UNSUPPORTED
