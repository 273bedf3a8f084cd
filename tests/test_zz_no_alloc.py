"""The allocation-free neighbor decode (lg_decode_neighbors_noalloc) against
lg_decode_neighbors, called through the C ABI: two calls in a row on each
graph and mode, the second with fewer vertices, must return exactly the
offsets and lists of the allocating entry point (and the input lists), and
the graph must hold no decode workspace afterwards.  Also the size limits and
the capacity error."""

import numpy as np
import pytest
import torch

from paper_2010_15879_amd import graphgen as gg

pytestmark = pytest.mark.gpu

ENCODINGS = [
    dict(layout="packed", ids="global", offsets="packed", relabel=False),
    dict(layout="packed", ids="local", offsets="succinct", relabel=True),
    dict(layout="packed", ids="local-gap", offsets="succinct", relabel=True),
    dict(layout="packed", ids="varint-diff", offsets="packed", relabel=True),
    dict(layout="plain", relabel="greedy"),
]


@pytest.fixture(scope="module")
def lgmod():
    from paper_2010_15879_amd import lg
    lg.lib()
    return lg


@pytest.fixture(scope="module")
def graph():
    g = gg.kronecker(13, 16, seed=9)
    print(f"[noalloc] kronecker s13: n={g.n} M={g.m}", flush=True)
    return g, g.to("cuda")


def reference(lg, h, vt, flags):
    off, ids = lg.decode_neighbors(h, vt, flags)
    return off.cpu().numpy(), ids.cpu().numpy()


@pytest.mark.parametrize("enc", ENCODINGS, ids=lambda e: "-".join(str(v) for v in e.values()))
@pytest.mark.parametrize("flags", ["sorted", "original", "raw"])
def test_noalloc_equals_allocating_decode(lgmod, graph, enc, flags):
    g, dg = graph
    off_h, col_h = g.numpy()
    print(f"[noalloc] {enc} {flags}", flush=True)
    h = lgmod.encode(dg.row_offsets, dg.col, g.n, **enc)
    bytes_before = h.info()["device_bytes"]
    rng = np.random.default_rng(5)
    # first call: 3,000 vertices (repeats allowed); second: 500 others
    for k in (3000, 500):
        vt = torch.from_numpy(rng.integers(0, g.n, size=k).astype(np.int32)).cuda()
        off = torch.empty(k + 1, dtype=torch.int64, device="cuda")
        ids = torch.full((int(g.m) + 1,), -7, dtype=torch.int32, device="cuda")
        st = lgmod.decode_neighbors_noalloc(h, vt, off, ids, flags)
        torch.cuda.synchronize()
        assert st == lgmod.LG_OK
        # the allocating entry point runs on another handle of the same graph,
        # so this one never gets a decode workspace
        h2 = lgmod.encode(dg.row_offsets, dg.col, g.n, **enc)
        want_off, want_ids = reference(lgmod, h2, vt, flags)
        h2.free()
        got_off = off.cpu().numpy()
        np.testing.assert_array_equal(got_off, want_off)
        total = int(got_off[-1])
        got = ids[:total].cpu().numpy()
        np.testing.assert_array_equal(got, want_ids)
        assert int(ids[total].item()) == -7  # nothing written past the lists
        if flags == "sorted":
            for i, v in enumerate(vt.cpu().numpy()):
                np.testing.assert_array_equal(got[got_off[i]:got_off[i + 1]], col_h[off_h[v]:off_h[v + 1]])
    assert h.info()["device_bytes"] == bytes_before
    h.free()


def test_noalloc_capacity_and_empty(lgmod, graph):
    g, dg = graph
    h = lgmod.encode(dg.row_offsets, dg.col, g.n, ids="local", offsets="succinct", relabel=True)
    vt = torch.arange(0, 256, dtype=torch.int32, device="cuda")
    off = torch.empty(257, dtype=torch.int64, device="cuda")
    small = torch.empty(3, dtype=torch.int32, device="cuda")
    st = lgmod.decode_neighbors_noalloc(h, vt, off, small, "sorted")
    assert st == lgmod.LG_ERR_CAPACITY
    want_off, _ = reference(lgmod, h, vt, "sorted")
    np.testing.assert_array_equal(off.cpu().numpy(), want_off)  # offsets written anyway
    off0 = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    assert lgmod.decode_neighbors_noalloc(h, empty, off0, small) == lgmod.LG_OK
    torch.cuda.synchronize()
    assert int(off0.item()) == 0
    h.free()


def test_noalloc_limits(lgmod):
    # more vertices than the limit: refused before any device work
    g = gg.kronecker(17, 16, seed=1)
    dg = g.to("cuda")
    h = lgmod.encode(dg.row_offsets, dg.col, g.n, ids="local", offsets="succinct", relabel=True)
    k = lgmod.LG_NOALLOC_MAX_VERTICES + 1
    vt = torch.zeros(k, dtype=torch.int32, device="cuda")
    off = torch.empty(k + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(lgmod.LGError) as ex:
        lgmod.decode_neighbors_noalloc(h, vt, off, ids, "sorted")
    assert ex.value.status == lgmod.LG_ERR_UNSUPPORTED and "LG_NOALLOC_MAX_VERTICES" in str(ex.value)
    # a sorted decode of more ids than the sort limit on a relabeled graph
    k = lgmod.LG_NOALLOC_MAX_VERTICES
    vt = torch.arange(0, k, dtype=torch.int32, device="cuda")
    off = torch.empty(k + 1, dtype=torch.int64, device="cuda")
    want_off, _ = reference(lgmod, h, vt, "sorted")
    assert int(want_off[-1]) > lgmod.LG_NOALLOC_MAX_SORTED_IDS
    ids = torch.empty(int(want_off[-1]), dtype=torch.int32, device="cuda")
    with pytest.raises(lgmod.LGError) as ex:
        lgmod.decode_neighbors_noalloc(h, vt, off, ids, "sorted")
    assert ex.value.status == lgmod.LG_ERR_UNSUPPORTED and "LG_NOALLOC_MAX_SORTED_IDS" in str(ex.value)
    np.testing.assert_array_equal(off.cpu().numpy(), want_off)
    # the same vertices in stored order need no sort and are served
    assert lgmod.decode_neighbors_noalloc(h, vt, off, ids, "original") == lgmod.LG_OK
    h.free()
