"""The query server on the GPU: every result served in a concurrent mix is
bit-exact with the same query served alone, and with the oracle; the budget
bounds the device bytes at every admission; queries that cannot fit are
rejected; batching of neighbor fetches happens under load."""

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


@pytest.fixture(scope="module")
def graphs(lgmod):
    """(CSR on the host, encoded handle) for four encodings of three graphs."""
    out = []
    specs = [
        (gg.kronecker(12, 16, seed=3), dict()),
        (gg.kronecker(12, 16, seed=3), dict(ids="local", offsets="succinct", relabel=True)),
        (gg.erdos_renyi(11, 8, seed=5), dict(ids="local")),
        (gg.kronecker(10, 16, seed=7), dict(layout="plain")),
    ]
    for g, kw in specs:
        gd = g.to("cuda")
        h = lgmod.encode(gd.row_offsets, gd.col, g.n, **kw)
        off, col = g.numpy()
        out.append((off.astype(np.uint64), col.view(np.uint32), h))
    return out


def make_queries(graphs, count, seed):
    """60% neighbor fetch, 30% 2-hop, 10% BFS; graph uniform; vertex uniform
    over the non-isolated vertices."""
    rng = np.random.default_rng(seed)
    qs = []
    for _ in range(count):
        gi = int(rng.integers(len(graphs)))
        off = graphs[gi][0]
        cand = np.nonzero(np.diff(off) > 0)[0]
        v = int(cand[rng.integers(cand.size)])
        r = rng.random()
        kind = "neighbors" if r < 0.6 else ("khop" if r < 0.9 else "bfs")
        qs.append((kind, gi, v))
    return qs


def run(srv, qs, one_at_a_time):
    res = []
    if one_at_a_time:
        for kind, gi, v in qs:
            t = srv.submit(kind, gi, v, k=2)
            res.append(srv.wait(t))
        return res
    tickets = [srv.submit(kind, gi, v, k=2) for kind, gi, v in qs]
    return [srv.wait(t) for t in tickets]


def same(a, b):
    assert a["status"] == b["status"] == 0
    assert a["count"] == b["count"]
    np.testing.assert_array_equal(a["ids"], b["ids"])
    assert a["digest"] == b["digest"] and a["max_depth"] == b["max_depth"]


def check_oracle(graphs, q, r):
    kind, gi, v = q
    off, col, _ = graphs[gi]
    if kind == "neighbors":
        np.testing.assert_array_equal(r["ids"], col[int(off[v]):int(off[v + 1])])
    else:
        d, _ = orc.bfs(off, col, v)
        if kind == "khop":
            np.testing.assert_array_equal(r["ids"], np.nonzero((d >= 1) & (d <= 2))[0])
        else:
            assert r["count"] == int(np.count_nonzero(d >= 0)) and r["max_depth"] == int(d.max())


def test_mix_equals_alone_and_oracle(lgmod, graphs):
    handles = [h for _, _, h in graphs]
    qs = make_queries(graphs, 400, seed=1)
    print("[serve] alone", flush=True)
    alone_srv = lgmod.Server(handles, workers=1)
    alone = run(alone_srv, qs, one_at_a_time=True)
    alone_srv.free()
    for q, r in zip(qs, alone):
        check_oracle(graphs, q, r)
    print("[serve] mix", flush=True)
    srv = lgmod.Server(handles, workers=8, max_batch=32)
    mix = run(srv, qs, one_at_a_time=False)
    st = srv.stats()
    srv.free()
    for a, b in zip(alone, mix):
        same(a, b)
    assert st["completed"] == st["submitted"] == len(qs) and st["rejected"] == 0
    assert st["overruns"] == 0
    # neighbor fetches queued together were served by shared launches
    assert st["batches"] < len(qs)
    assert max(r["batch"] for r in mix) > 1


def test_bfs_arrays_match_oracle(lgmod, graphs):
    srv = lgmod.Server([h for _, _, h in graphs], workers=4)
    tickets = []
    for gi, (off, col, _) in enumerate(graphs):
        v = int(np.nonzero(np.diff(off) > 0)[0][-1])
        tickets.append((gi, v, srv.submit("bfs", gi, v, keep_arrays=True)))
    for gi, v, t in tickets:
        r = srv.wait(t)
        off, col, h = graphs[gi]
        # parents: the smallest label among the candidates (the relabeled
        # graph labels by the degree ordering)
        d0, p0 = orc.bfs(off, col, v, relabeled=h.info()["relabel"] != 0)
        np.testing.assert_array_equal(r["depth"], d0)
        np.testing.assert_array_equal(r["parent"], p0)
    srv.free()


def test_tight_budget_serializes_and_holds(lgmod, graphs):
    handles = [h for _, _, h in graphs]
    resident = sum(h.info()["device_bytes"] for h in handles)
    n_max = max(h.n for h in handles)
    # room for about two BFS workspaces of the largest graph: admission must queue
    budget = resident + 2 * 80 * n_max
    qs = make_queries(graphs, 120, seed=2)
    srv = lgmod.Server(handles, budget_bytes=budget, workers=8)
    mix = run(srv, qs, one_at_a_time=False)
    st = srv.stats()
    srv.free()
    assert st["peak_bytes"] <= budget and st["overruns"] == 0
    assert st["resident_bytes"] == resident
    ok = [(q, r) for q, r in zip(qs, mix) if r["status"] == 0]
    assert len(ok) + st["rejected"] == len(qs)
    assert st["rejected"] == 0
    for q, r in ok:
        check_oracle(graphs, q, r)


def test_budget_rejections(lgmod, graphs):
    handles = [h for _, _, h in graphs]
    resident = sum(h.info()["device_bytes"] for h in handles)
    with pytest.raises(lgmod.LGError):
        lgmod.Server(handles, budget_bytes=resident - 1)
    srv = lgmod.Server(handles, budget_bytes=resident + 64, workers=2)
    t = srv.submit("bfs", 0, int(np.nonzero(np.diff(graphs[0][0]) > 0)[0][0]))
    r = srv.wait(t)
    assert r["status"] != 0
    st = srv.stats()
    assert st["rejected"] == 1 and st["peak_bytes"] <= resident + 64
    srv.free()
    with pytest.raises(lgmod.LGError):
        srv2 = lgmod.Server(handles)
        try:
            srv2.submit("neighbors", 0, graphs[0][2].n)  # vertex out of range
        finally:
            srv2.free()
