"""GPU parity at the benchmark's full size and launch configuration.

The bench workload (1,024 queries, eps = 1e-7, k = 50, on the 1M / 500k / 20M
graph with 10k attributes) runs through ahpp_query_batch exactly as bench.py
launches it.  Sampled queries are compared with the oracle's exact power
series (Def. 2, certified to 1e-12) element by element; every query is checked
through properties that hold at any size: the stop rule (max residue <=
eps/lambda), mass conservation (Lemma 2 summed over U), non-negativity and a
sorted, source-free top-k list.
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
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    _say("generate 1M/500k/20M graph")
    g = synth.make_graph("m1")
    _say("load")
    dg = ahpp.load_graph(g)
    yield g, dg, ahpp, torch
    dg.free()


@pytest.mark.timeout(900)
def test_bench_batch_matches_oracle(big):
    g, dg, ahpp, torch = big
    eps, k = 1e-7, 50
    srcs = synth.mixed_batch_queries(g, 1024, 2002)
    _say("batch of 1024 at eps 1e-7")
    res = ahpp.ahpp_query_batch(dg, srcs, eps, k=k)
    torch.cuda.synchronize()
    eps_f = eps / dg.lam
    tn = res.topk_n.cpu().numpy()
    tv = res.topk_val.cpu().numpy()
    ti = res.topk_idx.cpu().numpy()
    pis = res.pi
    sums = pis.double().sum(dim=1).cpu().numpy()
    mins = pis.min(dim=1).values.cpu().numpy()
    for q, st in enumerate(res.stats):
        assert st["converged"] == 1, q
        assert st["max_residual"] <= eps_f * (1 + 1e-6), q
        assert abs(sums[q] + st["sum_residual"] - 1.0) < 1e-5, (q, sums[q], st["sum_residual"])
        assert mins[q] >= 0.0
        assert tn[q] == k
        assert np.all(np.diff(tv[q]) <= 0) and int(srcs[q]) not in ti[q].tolist()
    og = O.OracleGraph.from_graph(g)
    for q in (0, 511, 512, 1023):
        s = int(srcs[q])
        _say("oracle power series for query", q, "source", s)
        exact, tail = og.power_series(s)
        assert tail < 1e-12
        pi = pis[q].cpu().numpy().astype(np.float64)
        chk = O.check_query(exact, pi, eps, tol=TOL, k=k, source=s, topk_ids=ti[q])
        assert chk.ok, (q, s, chk.detail)
        _say(f"query {q}: max |err| {chk.max_abs_err:.3e} = {chk.max_abs_err / eps:.3f} eps")


@pytest.mark.timeout(900)
def test_plain_query_matches_oracle(big):
    g, dg, ahpp, torch = big
    eps = 1e-7
    s = int(synth.degree_queries(g, 1, 2001)[0])
    _say("plain query", s)
    res = ahpp.ahpp_query(dg, s, eps, k=50, want_resid=True)
    exact, _ = O.OracleGraph.from_graph(g).power_series(s)
    chk = O.check_query(exact, res.pi.cpu().numpy().astype(np.float64), eps, tol=TOL,
                        resid=res.resid.cpu().numpy().astype(np.float64), k=50, source=s,
                        topk_ids=res.topk_idx[: int(res.topk_n.item())].cpu().numpy())
    assert chk.ok, chk.detail
