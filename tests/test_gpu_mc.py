"""Monte Carlo walks (Section 3.1, Lemma 1) against the oracle's exact rows.

Each node's stop count is Binomial(n_walks, pi(u, x)); every node must lie
within six standard deviations (plus 3 / n_walks for the rarest nodes) of
the exact value.  Walk accounting is exact: stops + lost + truncated walks
= n_walks.  Outputs depend only on the seed.
"""

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    return ahpp, torch


def _band_ok(exact, est, n):
    sd = np.sqrt(np.clip(exact * (1.0 - exact), 0.0, None) / n)
    dev = np.abs(est - exact)
    bad = dev > 6.0 * sd + 3.0 / n
    return (not bad.any()), (int(np.argmax(dev / (sd + 1.0 / n))) if bad.any() else -1)


def _walk_total(res, n):
    st = res["stats"]
    stops = int(round(float(res["pi"].double().sum().item()) * n))
    return stops + st["lost"] + st["truncated"]


def test_unit_graph_against_dense_solve(env, tiny_graph, tiny_Pi):
    ahpp, torch = env
    dg = ahpp.load_graph(tiny_graph)
    n = 4_000_000
    for s in synth.uniform_queries(tiny_graph, 2, 2000).tolist():
        _say("walks from", s)
        res = ahpp.ahpp_query_mc(dg, s, n, seed=7, k=20)
        est = res["pi"].cpu().numpy().astype(np.float64)
        ok, worst = _band_ok(tiny_Pi[s], est, n)
        assert ok, (s, worst, est[worst], tiny_Pi[s][worst])
        assert _walk_total(res, n) == n and res["stats"]["truncated"] == 0
        assert res["stats"]["lost"] == 0  # the generated graphs have no dangling U node
        # Top-k is the host order of the returned vector (source excluded).
        x = est.copy()
        x[s] = -np.inf
        order = np.lexsort((np.arange(x.size), -x))[:20]
        m = int(res["topk_n"].item())
        assert res["topk_idx"][:m].cpu().numpy().tolist() == [i for i in order.tolist() if x[i] > 0][:m]
    dg.free()


def test_weighted_graph_against_power_series(env):
    ahpp, torch = env
    g = synth.make_custom(5000, 2000, 40000, 200, 6, seed=919, unit_weights=False)
    og = O.OracleGraph.from_graph(g)
    dg = ahpp.load_graph(g)
    n = 8_000_000
    for s in synth.mixed_batch_queries(g, 2, 31).tolist():
        exact, _ = og.power_series(s)
        res = ahpp.ahpp_query_mc(dg, s, n, seed=11)
        est = res["pi"].cpu().numpy().astype(np.float64)
        ok, worst = _band_ok(exact, est, n)
        _say("source", s, "max |err|", float(np.abs(est - exact).max()), "steps", res["stats"]["steps"])
        assert ok, (s, worst, est[worst], exact[worst])
        # Mean walk length is (1 - alpha) / alpha steps of P.
        assert abs(res["stats"]["steps"] / n - 0.85 / 0.15) < 0.02
    dg.free()


def test_seed_determinism_and_dangling_loss(env):
    ahpp, torch = env
    # U node 3 has no edge and U node 4 no attribute: their steps of one kind lose the walk.
    eu = np.array([0, 0, 1, 2, 4, 1], np.int32)
    ev = np.array([0, 1, 1, 2, 0, 2], np.int32)
    au = np.array([0, 1, 2, 3, 3, 0], np.int32)
    aa = np.array([0, 0, 1, 1, 0, 1], np.int32)
    g = synth.AttributedBipartiteGraph(None, 5, 3, 2, eu, ev, np.ones(6, np.float32), au, aa,
                                       np.ones(6, np.float32))
    order = np.lexsort((aa, au))
    g.assoc_u, g.assoc_a = au[order], aa[order]
    og = O.OracleGraph.from_graph(g)
    dg = ahpp.load_graph(g)
    n = 2_000_000
    a = ahpp.ahpp_query_mc(dg, 0, n, seed=5)
    b = ahpp.ahpp_query_mc(dg, 0, n, seed=5)
    c = ahpp.ahpp_query_mc(dg, 0, n, seed=6)
    assert torch.equal(a["pi"], b["pi"]) and a["stats"] == {**b["stats"], "ms": a["stats"]["ms"]}
    assert not torch.equal(a["pi"], c["pi"])
    assert a["stats"]["lost"] > 0 and _walk_total(a, n) == n
    exact, _ = og.power_series(0)
    ok, worst = _band_ok(exact, a["pi"].cpu().numpy().astype(np.float64), n)
    assert ok, worst
    # The lost share equals the mass the exact series loses.
    assert abs(a["stats"]["lost"] / n - (1.0 - exact.sum())) < 6.0 * np.sqrt(0.25 / n)
    dg.free()


def test_walk_count_limits(env):
    """Stop counts are 32-bit: n_walks outside [1, 2^32 - 1] is refused before
    any walk runs."""
    ahpp, torch = env
    g = synth.make_graph("tiny")
    dg = ahpp.load_graph(g, device=0)
    try:
        for n in (0, 2 ** 32, 2 ** 40):
            _say("walk count limit", n)
            with pytest.raises(ahpp.AhppError) as e:
                ahpp.ahpp_query_mc(dg, 3, n, seed=1)
            assert e.value.status == -1
        res = ahpp.ahpp_query_mc(dg, 3, 1000, seed=1)
        assert res["stats"]["walks"] == 1000
    finally:
        dg.free()
