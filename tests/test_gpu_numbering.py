"""The device renumbers U, V and the attributes by reference count and maps
sources in and scores out.  Relabelling a graph's nodes by random
permutations must not change the answer: the scores of a source on the
relabelled graph, mapped back, equal those on the original up to float
rounding (the two graphs may order tied nodes differently), and each top-k
passes the oracle's band check in its own numbering.  Covers the plain
query, the batch and the server."""

import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6
EPS = 1e-7


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    g = synth.make_custom(4000, 1500, 30000, 150, 5, seed=520, unit_weights=False)
    rng = np.random.default_rng(20)
    pu, pv, pa = (rng.permutation(n).astype(np.int32) for n in (g.n_u, g.n_v, g.n_attr))
    h = dataclasses.replace(g, edge_u=pu[g.edge_u], edge_v=pv[g.edge_v], assoc_u=pu[g.assoc_u],
                            assoc_a=pa[g.assoc_a])
    dg, dh = ahpp.load_graph(g), ahpp.load_graph(h)
    yield ahpp, torch, g, h, pu, dg, dh, O.OracleGraph.from_graph(g)
    dg.free()
    dh.free()


def _topk_ok(exact, ids, s, k=20):
    return O.topk_band_ok(exact, ids, k, EPS + TOL, s)


def test_plain_query_is_label_free(env):
    ahpp, torch, g, h, pu, dg, dh, og = env
    assert abs(dg.lam - dh.lam) <= 1e-6 * dg.lam
    for s in synth.mixed_batch_queries(g, 4, 21).tolist():
        exact, _ = og.power_series(s)
        a = ahpp.ahpp_query(dg, s, EPS, k=20, want_resid=True)
        b = ahpp.ahpp_query(dh, int(pu[s]), EPS, k=20, want_resid=True)
        pa_, pb_ = a.pi.cpu().numpy(), b.pi.cpu().numpy()[pu]
        assert np.abs(pa_.astype(np.float64) - pb_).max() <= 1e-7
        assert np.abs(a.resid.cpu().numpy() - b.resid.cpu().numpy()[pu]).max() <= 1e-7
        assert abs(a.stats[0]["iters"] - b.stats[0]["iters"]) <= 1
        assert _topk_ok(exact, a.topk_idx[: int(a.topk_n.item())].cpu().numpy(), s)
        assert _topk_ok(exact[np.argsort(pu)], b.topk_idx[: int(b.topk_n.item())].cpu().numpy(), int(pu[s]))
        assert int(pu[s]) not in b.topk_idx[: int(b.topk_n.item())].cpu().numpy().tolist()


def test_batch_and_server_are_label_free(env):
    ahpp, torch, g, h, pu, dg, dh, og = env
    srcs = synth.mixed_batch_queries(g, 300, 22)
    a = ahpp.ahpp_query_batch(dg, srcs, EPS, k=20)
    b = ahpp.ahpp_query_batch(dh, pu[srcs], EPS, k=20)
    pa_ = a.pi.cpu().numpy()
    pb_ = b.pi.cpu().numpy()[:, pu]
    assert np.abs(pa_.astype(np.float64) - pb_).max() <= 1e-7
    for q in (0, 150, 299):
        s = int(srcs[q])
        exact, _ = og.power_series(s)
        ids = b.topk_idx[q, : int(b.topk_n[q].item())].cpu().numpy()
        assert _topk_ok(exact[np.argsort(pu)], ids, int(pu[s]))
    srv = ahpp.Server(dh, k=20, max_slots=256, keep_pi=True)
    for t, s in enumerate(srcs[:40].tolist()):
        srv.submit(t, int(pu[s]), EPS)
    got = {}
    for _ in range(2000):
        srv.step(8)
        for r in srv.results(want_pi=True):
            got[r["tag"]] = r
        if len(got) == 40:
            break
    srv.close()
    assert len(got) == 40
    for t in (0, 17, 39):
        assert np.abs(got[t]["pi"].cpu().numpy()[pu].astype(np.float64) - pa_[t]).max() <= 1e-7
