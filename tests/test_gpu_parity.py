"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Acceptance per query (Theorem 2 with the tolerance of the GPU's float32
arithmetic): |pi - pi_hat| <= eps + 1e-6, pi_hat >= 0, pi_hat <= pi + 1e-6,
|sum pi_hat + sum r - 1| <= 1e-5 without dangling nodes, and the top-k list
inside the band around the exact k-th score.  Index work (top-k of a given
vector) is compared exactly.
"""

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ahpp(torch_cuda):
    from paper_2512_11606_amd import ahpp as A
    A.load_library()
    return A


@pytest.fixture(scope="module")
def tiny(ahpp, tiny_graph):
    _say("load tiny graph")
    g = ahpp.load_graph(tiny_graph)
    yield g
    g.free()


def _check(torch, res, exact, eps, k=0, source=-1, resid=True):
    pi = res.pi.cpu().numpy().astype(np.float64)
    r = res.resid.cpu().numpy().astype(np.float64) if (resid and res.resid is not None) else None
    ids = res.topk_idx[: int(res.topk_n.item())].cpu().numpy() if k else None
    return O.check_query(exact, pi, eps, tol=TOL, resid=r, k=k, source=source, topk_ids=ids)


def test_lambda_matches_theorem3(tiny, tiny_oracle):
    lam_o = tiny_oracle.lambda_thm3(T=tiny.info["lambda_iters"])
    assert tiny.lam >= lam_o
    assert tiny.lam == pytest.approx(lam_o * (1 + 1e-4), rel=2e-5)


def test_graph_info(tiny, tiny_graph):
    i = tiny.info
    assert (i["n_u"], i["n_v"], i["n_attr"]) == (tiny_graph.n_u, tiny_graph.n_v, tiny_graph.n_attr)
    assert i["n_edges"] == tiny_graph.m_e and i["n_assoc"] == tiny_graph.m_a
    assert i["dangling_u"] == 0


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_tiny_queries_meet_guarantee(torch_cuda, ahpp, tiny, tiny_Pi, tiny_graph, eps):
    srcs = synth.uniform_queries(tiny_graph, 40, 4242)
    srcs = np.concatenate([srcs, synth.hub_queries(tiny_graph, 8, 4243)])
    worst = 0.0
    for s in srcs.tolist():
        _say("tiny query", s, eps)
        res = ahpp.ahpp_query(tiny, s, eps, k=20, want_resid=True)
        chk = _check(torch_cuda, res, tiny_Pi[s], eps, k=20, source=s)
        assert chk.ok, (s, chk.detail)
        assert res.stats[0]["converged"] == 1
        assert res.stats[0]["max_residual"] <= eps / tiny.lam * (1 + 1e-6)
        worst = max(worst, chk.max_abs_err)
    print(f"worst |err| = {worst:.3e} (eps {eps:g})")


def test_weighted_graph_against_power_series(torch_cuda, ahpp):
    g = synth.make_custom(6000, 2500, 60000, 300, 8, seed=515, unit_weights=False)
    og = O.OracleGraph.from_graph(g)
    _say("load weighted 6000-node graph")
    dg = ahpp.load_graph(g)
    lam_o = og.lambda_thm3(T=dg.info["lambda_iters"])
    assert dg.lam == pytest.approx(lam_o * (1 + 1e-4), rel=2e-5)
    for s in synth.degree_queries(g, 6, 99).tolist():
        for eps in (1e-5, 1e-7):
            _say("weighted query", s, eps)
            res = ahpp.ahpp_query(dg, s, eps, k=50, want_resid=True)
            exact, _ = og.power_series(s)
            chk = _check(torch_cuda, res, exact, eps, k=50, source=s)
            assert chk.ok, (s, eps, chk.detail)
    dg.free()


@pytest.mark.parametrize("mode", ["nodes", "edges"])
def test_sampled_graph_against_power_series(torch_cuda, ahpp, mode):
    """Exp-3's sampled graphs (attributes without members, renumbered ids):
    plain and batched queries against the exact series."""
    g = synth.sample_graph(synth.make_custom(6000, 2500, 60000, 300, 8, seed=516, unit_weights=False), 0.6, mode,
                           seed=7)
    og = O.OracleGraph.from_graph(g)
    dg = ahpp.load_graph(g)
    srcs = synth.degree_queries(g, 3, 98)
    _say("sampled graph", mode, g.n_u, g.n_v, g.m_e, g.m_a)
    batch = ahpp.ahpp_query_batch(dg, srcs, 1e-6, k=30)
    for q, s in enumerate(srcs.tolist()):
        exact, _ = og.power_series(s)
        chk = _check(torch_cuda, ahpp.ahpp_query(dg, s, 1e-6, k=30, want_resid=True), exact, 1e-6, k=30, source=s)
        assert chk.ok, (mode, s, chk.detail)
        chk = O.check_query(exact, batch.pi[q].cpu().numpy().astype(np.float64), 1e-6, k=30, source=s,
                            topk_ids=batch.topk_idx[q, : int(batch.topk_n[q].item())].cpu().numpy())
        assert chk.ok, (mode, s, "batched", chk.detail)
    og.close()
    dg.free()


def test_edgeless_v_nodes_change_nothing(torch_cuda, ahpp):
    """V nodes without an edge (before, between and after the others) are
    dropped at load: the scores equal, bit for bit, those of the same graph
    numbered without them, and the graph info keeps the caller's V count."""
    import dataclasses
    g = synth.make_custom(3000, 1200, 25000, 100, 5, seed=517, unit_weights=False)
    spread = dataclasses.replace(g, n_v=3 * g.n_v + 2, edge_v=(3 * g.edge_v + 1).astype(np.int32))
    a, b = ahpp.load_graph(g), ahpp.load_graph(spread)
    assert b.info["n_v"] == 3 * g.n_v + 2 and a.lam == b.lam
    srcs = synth.degree_queries(g, 3, 97)
    for s in srcs.tolist():
        ra, rb = ahpp.ahpp_query(a, s, 1e-7, k=20), ahpp.ahpp_query(b, s, 1e-7, k=20)
        assert torch_cuda.equal(ra.pi, rb.pi) and torch_cuda.equal(ra.topk_idx, rb.topk_idx)
    ba, bb = ahpp.ahpp_query_batch(a, srcs, 1e-7, k=20), ahpp.ahpp_query_batch(b, srcs, 1e-7, k=20)
    assert torch_cuda.equal(ba.pi, bb.pi)
    exact, _ = O.OracleGraph.from_graph(spread).power_series(int(srcs[0]))
    assert _check(torch_cuda, ahpp.ahpp_query(b, int(srcs[0]), 1e-7, want_resid=True), exact, 1e-7).ok
    a.free()
    b.free()


@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_pure_structure_and_pure_attribute_walks(torch_cuda, ahpp, tiny_graph, beta):
    og = O.OracleGraph.from_graph(tiny_graph)
    _say("load tiny beta", beta)
    dg = ahpp.load_graph(tiny_graph, beta=beta)
    for s in (3, 1000):
        res = ahpp.ahpp_query(dg, s, 1e-6, k=10, want_resid=True)
        exact, _ = og.power_series(s, beta=beta)
        chk = _check(torch_cuda, res, exact, 1e-6, k=10, source=s)
        assert chk.ok, chk.detail
    dg.free()


def test_topk_exact_on_given_vector(torch_cuda, ahpp, tiny):
    torch = torch_cuda
    rng = np.random.default_rng(7)
    n = tiny.n_u
    for trial in range(4):
        v = (rng.integers(0, 9, size=n) / 7.0).astype(np.float32)  # many ties and zeros
        if trial == 3:
            v[:] = 0
            v[[5, 9, 700]] = [0.5, 0.5, 0.25]
        t = torch.from_numpy(v).cuda()
        for k, ex in ((1, -1), (20, 5), (333, 17), (2048, -1)):
            _say("topk trial", trial, k, ex)
            ti, tv, tn = ahpp.ahpp_topk(tiny, t, k, ex)
            torch.cuda.synchronize()
            ids, vals = O.topk(v.astype(np.float64), k, ex)
            m = int(tn.item())
            assert m == len(ids)
            assert ti[:m].cpu().numpy().tolist() == ids.tolist()
            assert np.array_equal(tv[:m].cpu().numpy(), vals.astype(np.float32))


def test_batch_equals_alone(torch_cuda, ahpp, tiny, tiny_Pi, tiny_graph):
    srcs = synth.mixed_batch_queries(tiny_graph, 24, 2002)
    eps = np.array([1e-4, 1e-6, 1e-5, 1e-7] * 6)
    _say("batch of", len(srcs))
    res = ahpp.ahpp_query_batch(tiny, srcs, eps, k=20)
    pis = res.pi.cpu().numpy()
    for q, s in enumerate(srcs.tolist()):
        chk = O.check_query(tiny_Pi[s], pis[q].astype(np.float64), eps[q], tol=TOL, k=20, source=s,
                            topk_ids=res.topk_idx[q, : int(res.topk_n[q].item())].cpu().numpy())
        assert chk.ok, (q, s, chk.detail)
        alone = ahpp.ahpp_query(tiny, s, float(eps[q]))
        assert np.abs(alone.pi.cpu().numpy() - pis[q]).max() <= eps[q] + TOL


def test_edge_cases(torch_cuda, ahpp):
    # A U node with no edge and no attribute (dangling), an attribute-only node,
    # a graph with no V side at all, and eps so large nothing is pushed.
    edges = [(0, 0), (1, 0), (1, 1), (2, 1)]
    assoc = [(0, 0), (1, 0), (3, 1), (2, 1)]
    import types
    e = np.array(edges, dtype=np.int32)
    a = np.array(assoc, dtype=np.int32)
    g = types.SimpleNamespace(n_u=5, n_v=2, n_attr=2, edge_u=e[:, 0], edge_v=e[:, 1],
                              edge_w=np.array([1, 2, 0.5, 1], np.float32), assoc_u=a[:, 0], assoc_a=a[:, 1],
                              assoc_w=np.array([1, 1, 3, 0.25], np.float32))
    og = O.OracleGraph.from_graph(g)
    _say("edge-case graph")
    dg = ahpp.load_graph(g)
    assert dg.info["dangling_u"] == 2  # node 3 (no edge) and node 4 (nothing)
    Pi = O.exact_dense(g)
    for s in range(5):
        res = ahpp.ahpp_query(dg, s, 1e-7, k=3, want_resid=True)
        chk = _check(torch_cuda, res, Pi[s], 1e-7, k=3, source=s, resid=False)
        assert chk.ok, (s, chk.detail)
    # eps >= lambda: the stop rule holds before any push, pi_hat = 0.
    res = ahpp.ahpp_query(dg, 0, 10.0 * dg.lam, k=2)
    assert float(res.pi.abs().max()) == 0.0 and int(res.topk_n.item()) == 0
    assert res.stats[0]["iters"] == 0
    dg.free()
    # Attributes only (no edges).
    g2 = types.SimpleNamespace(n_u=4, n_v=0, n_attr=2, edge_u=np.zeros(0, np.int32), edge_v=np.zeros(0, np.int32),
                               edge_w=None, assoc_u=np.array([0, 1, 2, 3, 0], np.int32),
                               assoc_a=np.array([0, 0, 1, 1, 1], np.int32), assoc_w=None)
    dg2 = ahpp.load_graph(g2, beta=1.0)
    Pi2 = O.exact_dense(g2, beta=1.0)
    for s in range(4):
        res = ahpp.ahpp_query(dg2, s, 1e-7, want_resid=True)
        chk = _check(torch_cuda, res, Pi2[s], 1e-7)
        assert chk.ok, chk.detail
    dg2.free()


def test_batch_edge_cases(torch_cuda, ahpp):
    """The batched engine on the same degenerate graphs: dangling U nodes, an
    attribute-only node, a graph with no V side; a query whose eps is at
    least lambda stops before any push inside a batch of running ones; an
    empty batch is a no-op."""
    import types
    e = np.array([(0, 0), (1, 0), (1, 1), (2, 1)], dtype=np.int32)
    a = np.array([(0, 0), (1, 0), (3, 1), (2, 1)], dtype=np.int32)
    g = types.SimpleNamespace(n_u=5, n_v=2, n_attr=2, edge_u=e[:, 0], edge_v=e[:, 1],
                              edge_w=np.array([1, 2, 0.5, 1], np.float32), assoc_u=a[:, 0], assoc_a=a[:, 1],
                              assoc_w=np.array([1, 1, 3, 0.25], np.float32))
    dg = ahpp.load_graph(g)
    Pi = O.exact_dense(g)
    _say("edge-case graph, batched")
    srcs = np.array([0, 1, 2, 3, 4, 0], dtype=np.int64)
    eps = np.array([1e-7] * 5 + [10.0 * dg.lam])
    res = ahpp.ahpp_query_batch(dg, srcs, eps, k=3)
    pis = res.pi.cpu().numpy().astype(np.float64)
    for q in range(5):
        s = int(srcs[q])
        chk = O.check_query(Pi[s], pis[q], 1e-7, tol=TOL, k=3, source=s,
                            topk_ids=res.topk_idx[q, : int(res.topk_n[q].item())].cpu().numpy())
        assert chk.ok, (s, chk.detail)
    assert float(np.abs(pis[5]).max()) == 0.0 and int(res.topk_n[5].item()) == 0
    assert res.stats[5]["iters"] == 0 and res.stats[5]["converged"] == 1
    empty = ahpp.ahpp_query_batch(dg, np.zeros(0, dtype=np.int64), 1e-7, k=3)
    assert empty.pi.shape == (0, 5) and empty.stats == []
    dg.free()
    g2 = types.SimpleNamespace(n_u=4, n_v=0, n_attr=2, edge_u=np.zeros(0, np.int32), edge_v=np.zeros(0, np.int32),
                               edge_w=None, assoc_u=np.array([0, 1, 2, 3, 0], np.int32),
                               assoc_a=np.array([0, 0, 1, 1, 1], np.int32), assoc_w=None)
    dg2 = ahpp.load_graph(g2, beta=1.0)
    Pi2 = O.exact_dense(g2, beta=1.0)
    _say("attribute-only graph, batched")
    res = ahpp.ahpp_query_batch(dg2, np.arange(4), 1e-7)
    pis = res.pi.cpu().numpy().astype(np.float64)
    for s in range(4):
        chk = O.check_query(Pi2[s], pis[s], 1e-7, tol=TOL)
        assert chk.ok, (s, chk.detail)
    dg2.free()


def test_errors(torch_cuda, ahpp, tiny, tiny_graph):
    with pytest.raises(ahpp.AhppError) as e:
        ahpp.ahpp_query(tiny, tiny.n_u, 1e-6)
    assert e.value.status == ahpp.ERR_INVALID_ARG
    with pytest.raises(ahpp.AhppError):
        ahpp.ahpp_query(tiny, 0, 0.0)
    with pytest.raises(ahpp.AhppError):
        ahpp.ahpp_query(tiny, 0, 1e-6, k=5000)
    with pytest.raises(ahpp.AhppError) as e:
        ahpp.ahpp_query(tiny, 0, 1e-6, max_iters=1)
    assert e.value.status == ahpp.ERR_NOT_CONVERGED
    res = ahpp.ahpp_query(tiny, 0, 1e-6, max_iters=1, allow_not_converged=True)
    assert res.stats[0]["iters"] == 1 and res.stats[0]["converged"] == 0
    bad_v = tiny_graph.edge_v.copy()
    bad_v[3] = tiny_graph.n_v
    with pytest.raises(ahpp.AhppError) as e:
        ahpp.ahpp_graph_load(tiny_graph.n_u, tiny_graph.n_v, tiny_graph.n_attr, tiny_graph.edge_u, bad_v,
                             tiny_graph.edge_w, tiny_graph.assoc_u, tiny_graph.assoc_a, tiny_graph.assoc_w)
    assert e.value.status == ahpp.ERR_INVALID_ARG and "edge id" in str(e.value)
    bad_w = tiny_graph.assoc_w.copy()
    bad_w[0] = 0.0
    with pytest.raises(ahpp.AhppError):
        ahpp.ahpp_graph_load(tiny_graph.n_u, tiny_graph.n_v, tiny_graph.n_attr, tiny_graph.edge_u, tiny_graph.edge_v,
                             tiny_graph.edge_w, tiny_graph.assoc_u, tiny_graph.assoc_a, bad_w)


def test_batch_weighted_ragged_tiles(torch_cuda, ahpp, monkeypatch):
    """Batches spanning several 256-query tiles with a ragged last tile, mixed
    eps; the same batch run one tile per pass gives bitwise the same result
    (every query's arithmetic is independent of its tile and lane)."""
    g = synth.make_custom(5000, 2000, 40000, 200, 6, seed=616, unit_weights=False)
    og = O.OracleGraph.from_graph(g)
    _say("load weighted 5000-node graph for batches")
    dg = ahpp.load_graph(g)
    assert dg.info["hot_rows"] == 8
    srcs = np.concatenate([synth.mixed_batch_queries(g, 400, 31), synth.degree_queries(g, 200, 32)])
    eps = np.where(np.arange(srcs.size) % 3 == 0, 1e-7, np.where(np.arange(srcs.size) % 3 == 1, 1e-5, 1e-6))
    _say("batch of", srcs.size)
    res = ahpp.ahpp_query_batch(dg, srcs, eps, k=25)
    pis = res.pi.cpu().numpy()
    for q in range(0, srcs.size, 11):
        s = int(srcs[q])
        exact, _ = og.power_series(s)
        chk = O.check_query(exact, pis[q].astype(np.float64), eps[q], tol=TOL, k=25, source=s,
                            topk_ids=res.topk_idx[q, : int(res.topk_n[q].item())].cpu().numpy())
        assert chk.ok, (q, s, chk.detail)
        st = res.stats[q]
        assert st["converged"] == 1 and st["max_residual"] <= eps[q] / dg.lam * (1 + 1e-6)
        assert abs(float(pis[q].sum()) + st["sum_residual"] - 1) < 1e-5
    # Same queries alone: results agree within the guarantee.
    for q in (0, 255, 256, 599):
        alone = ahpp.ahpp_query(dg, int(srcs[q]), float(eps[q])).pi.cpu().numpy()
        assert np.abs(alone - pis[q]).max() <= eps[q] + TOL
    # One tile in flight: three passes instead of one, identical bits.
    monkeypatch.setenv("AHPP_BATCH_TILES", "1")
    _say("same batch, one tile per pass")
    res1 = ahpp.ahpp_query_batch(dg, srcs, eps, k=25)
    assert np.array_equal(res1.pi.cpu().numpy(), pis)
    assert np.array_equal(res1.topk_idx.cpu().numpy(), res.topk_idx.cpu().numpy())
    assert [s["iters"] for s in res1.stats] == [s["iters"] for s in res.stats]
    dg.free()


def _hot_small_graph(n_u, seed):
    """V node 0 and attribute 0 link every U node ceil(1024 / n_u) + 1 times
    (repeated pairs, R12), so both rows pass 1,024 entries and become hot
    rows; other edges and attributes are random, weights in [0.5, 1) and
    (0, 1]."""
    import types
    rng = np.random.default_rng(seed)
    n_v, n_a = 12, 6
    rep = -(-1024 // n_u) + 1
    allu = np.repeat(np.arange(n_u), rep)
    m, ma = 6 * n_u, 3 * n_u
    edge_u = np.concatenate([allu, rng.integers(0, n_u, m)]).astype(np.int32)
    edge_v = np.concatenate([np.zeros(allu.size), rng.integers(1, n_v, m)]).astype(np.int32)
    assoc_u = np.concatenate([allu, rng.integers(0, n_u, ma)]).astype(np.int32)
    assoc_a = np.concatenate([np.zeros(allu.size), rng.integers(1, n_a, ma)]).astype(np.int32)
    return types.SimpleNamespace(
        n_u=n_u, n_v=n_v, n_attr=n_a, edge_u=edge_u, edge_v=edge_v,
        edge_w=rng.uniform(0.5, 1.0, edge_u.size).astype(np.float32),
        assoc_u=assoc_u, assoc_a=assoc_a, assoc_w=(1.0 - rng.random(assoc_u.size)).astype(np.float32))


@pytest.mark.parametrize("n_u", [20, 33, 70])
def test_hot_rows_over_small_u(torch_cuda, ahpp, monkeypatch, n_u):
    """Hot rows over a U smaller than one 32-node stage of the dense pass, one
    node past it, and a few stages with a ragged end (the pass masks the U
    rows past n_U and the weight block is zero past them).  Every source's
    batched answer meets Theorem 2 against the oracle's exact series, and so
    does the same graph loaded without hot rows (AHPP_HOT_ROWS=0)."""
    g = _hot_small_graph(n_u, 900 + n_u)
    og = O.OracleGraph.from_graph(g)
    srcs = np.arange(n_u, dtype=np.int64)
    exact = [og.power_series(int(s))[0] for s in srcs]
    for hot, want in (("128", 2), ("0", 0)):
        monkeypatch.setenv("AHPP_HOT_ROWS", hot)
        dg = ahpp.load_graph(g)
        assert dg.info["hot_rows"] == want, dg.info
        _say("small-U batch", n_u, "hot rows", want)
        res = ahpp.ahpp_query_batch(dg, srcs, 1e-7, k=10)
        pis = res.pi.cpu().numpy()
        for q, s in enumerate(srcs.tolist()):
            chk = O.check_query(exact[q], pis[q].astype(np.float64), 1e-7, tol=TOL, k=10, source=s,
                                topk_ids=res.topk_idx[q, : int(res.topk_n[q].item())].cpu().numpy())
            assert chk.ok, (n_u, hot, s, chk.detail)
            assert res.stats[q]["converged"] == 1
        dg.free()
    og.close()


def test_captured_rounds_match_plain_launches(torch_cuda, ahpp, tiny, tiny_graph, monkeypatch):
    """Rounds replayed from HIP graphs give bitwise the results of plain
    launches: single queries and a two-tile batch, replayed three times with
    unrelated eager GPU work and synchronisations between the replays."""
    import torch
    srcs = synth.mixed_batch_queries(tiny_graph, 300, 77)
    eps = np.array([(1e-4, 1e-6, 1e-7)[i % 3] for i in range(srcs.size)])
    monkeypatch.setenv("AHPP_GRAPHS", "0")
    ref_single = [ahpp.ahpp_query(tiny, int(s), 1e-6, k=20) for s in srcs[:3]]
    ref_batch = ahpp.ahpp_query_batch(tiny, srcs, eps, k=20)
    monkeypatch.setenv("AHPP_GRAPHS", "1")
    for rep in range(3):
        _say("graph replay", rep)
        for i, s in enumerate(srcs[:3]):
            r = ahpp.ahpp_query(tiny, int(s), 1e-6, k=20)
            assert torch.equal(r.pi, ref_single[i].pi), (rep, i)
            assert r.stats[0]["iters"] == ref_single[i].stats[0]["iters"]
        res = ahpp.ahpp_query_batch(tiny, srcs, eps, k=20)
        assert torch.equal(res.pi, ref_batch.pi), rep
        assert torch.equal(res.topk_idx, ref_batch.topk_idx), rep
        x = torch.randn(4096, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert torch.isfinite(x).all()


def test_tuned_schedule_changes_speed_only(torch_cuda, ahpp, monkeypatch):
    """The autotuner picks a schedule among its candidates; batch results are
    bitwise the same before and after, and with 1 or 4 tiles in flight (every
    sum has a fixed order, the hot rows' chunk partials included: this graph
    has 8 rows of over 1,024 entries, and its U spans several 32-node stages
    per chunk)."""
    import torch
    g = synth.make_custom(6000, 3000, 60000, 300, 6, seed=818, unit_weights=False)
    dg = ahpp.load_graph(g)
    assert dg.info["hot_rows"] == 8
    srcs = np.concatenate([synth.mixed_batch_queries(g, 800, 51), synth.degree_queries(g, 100, 52)])
    eps = np.where(np.arange(srcs.size) % 2 == 0, 1e-6, 1e-7)
    before = ahpp.ahpp_query_batch(dg, srcs, eps, k=25)
    info = ahpp.ahpp_graph_tune(dg, max_tiles=4)
    _say("tuned", info)
    assert info["tiles_in_flight"] in (1, 2, 4) and info["workgroup_multiplier"] in (1, 2, 4, 8)
    assert info["candidates"] >= 3 and 0 < info["ms_per_tile_round"] <= info["default_ms_per_tile_round"] * 1.0001
    after = ahpp.ahpp_query_batch(dg, srcs, eps, k=25)
    assert torch.equal(before.pi, after.pi)
    assert torch.equal(before.topk_idx, after.topk_idx)
    assert [s["iters"] for s in before.stats] == [s["iters"] for s in after.stats]
    for tiles in ("1", "4"):
        monkeypatch.setenv("AHPP_BATCH_TILES", tiles)
        _say("same batch,", tiles, "tiles in flight")
        res = ahpp.ahpp_query_batch(dg, srcs, eps, k=25)
        assert torch.equal(before.pi, res.pi), tiles
        assert torch.equal(before.topk_idx, res.topk_idx), tiles
    dg.free()
