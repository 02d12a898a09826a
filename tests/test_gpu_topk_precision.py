"""Exp-6's top-k precision on the 1M / 500k / 20M graph: for k = 200, 400,
600 at eps = 1e-6, the share of the exact top-k (the oracle's power series,
tail below 1e-12) that the device's top-k finds, for the plain ASRP query,
the batched one and the APP / APP(E) schedules.  Every device top-600 also
passes the band check, which holds for any eps-approximate vector: every
node whose exact score is more than 2 (eps + 1e-6) above the 600th exact
score is returned, none that far below it is; the precision itself is a
measured statistic, printed, with a floor of 0.9."""

import time

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6
KS = (200, 400, 600)


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _exact_topk(x, k, source):
    x = x.copy()
    x[source] = -np.inf
    return np.lexsort((np.arange(x.size), -x))[:k]


@pytest.mark.timeout(600)
def test_topk_precision_on_m1():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    g = synth.make_graph("m1")
    dg = ahpp.load_graph(g)
    og = O.OracleGraph.from_graph(g)
    srcs = synth.degree_queries(g, 3, 2009)
    kmax = max(KS)
    batch = ahpp.ahpp_query_batch(dg, srcs, EPS, k=kmax, want_pi=False)
    prec = {}
    for q, s in enumerate(srcs.tolist()):
        t0 = time.time()
        exact, tail = og.power_series(s)
        _say(f"source {s}: exact series in {time.time() - t0:.1f} s, tail {tail:.1e}")
        runs = {"ASRP": ahpp.ahpp_query(dg, s, EPS, k=kmax),
                "APP": ahpp.ahpp_query_schedule(dg, s, EPS, 1, k=kmax),
                "APP(E)": ahpp.ahpp_query_schedule(dg, s, EPS, 3, k=kmax)}
        tops = {name: r.topk_idx[: int(r.topk_n.item())].cpu().numpy() for name, r in runs.items()}
        tops["ASRP batched"] = batch.topk_idx[q, : int(batch.topk_n[q].item())].cpu().numpy()
        for name, r in runs.items():
            chk = O.check_query(exact, r.pi.cpu().numpy().astype(np.float64), EPS, k=kmax, source=s,
                                topk_ids=tops[name])
            assert chk.ok, (name, s, chk.detail)
        for k in KS:
            want = set(_exact_topk(exact, k, s).tolist())
            for name, top in tops.items():
                assert top.size >= k, (name, s, top.size)
                p = len(want & set(top[:k].tolist())) / k
                prec.setdefault((name, k), []).append(p)
    og.close()
    dg.free()
    for (name, k), ps in sorted(prec.items()):
        _say(f"precision {name} k={k}: mean {np.mean(ps):.4f} min {min(ps):.4f}")
        assert min(ps) >= 0.9, (name, k, ps)
