"""Metamorphic properties of the HIP path through the C ABI.

* Eq. 1 and Eq. 2 are scale-free in each weight kind; scaling by powers of two
  is exact in float32, so the device scores, residues and top-k lists of the
  scaled graph equal those of the original bit for bit (the single query and
  the batch).
* A pair listed twice with half the weight each is the pair listed once: the
  device answer on the split graph meets Theorem 2 against the exact series of
  the original graph.
* Walks stay in their component: on the disjoint union of two graphs a query
  leaves every score and residue of the other component exactly zero, alone,
  in a batch that mixes sources of both components, under Exp-2's other
  schedules and with the Monte Carlo estimator.
The Monte Carlo walks keep the first two properties as well: bit for bit
under power-of-two scaling with the same seed, and within the binomial band
of the unsplit graph's exact row on the split one.
"""

import types

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    ahpp.load_library()
    return torch, ahpp


def _ns(g, **kw):
    f = dict(n_u=g.n_u, n_v=g.n_v, n_attr=g.n_attr, edge_u=g.edge_u, edge_v=g.edge_v, edge_w=g.edge_w,
             assoc_u=g.assoc_u, assoc_a=g.assoc_a, assoc_w=g.assoc_w)
    f.update(kw)
    return types.SimpleNamespace(**f)


def test_power_of_two_scaling_is_bitwise(env):
    torch, A = env
    g = synth.make_custom(5000, 2000, 45000, 200, 6, seed=611, unit_weights=False)
    h = _ns(g, edge_w=(g.edge_w * np.float32(4)).astype(np.float32),
            assoc_w=(g.assoc_w * np.float32(0.5)).astype(np.float32))
    _say("scaled graphs", g.n_u, g.m_e, g.m_a)
    a, b = A.load_graph(g), A.load_graph(h)
    assert a.lam == b.lam
    srcs = synth.degree_queries(g, 4, 612)
    for s in srcs.tolist():
        ra = A.ahpp_query(a, s, 1e-7, k=40, want_resid=True)
        rb = A.ahpp_query(b, s, 1e-7, k=40, want_resid=True)
        assert torch.equal(ra.pi, rb.pi) and torch.equal(ra.resid, rb.resid), s
        assert torch.equal(ra.topk_idx, rb.topk_idx) and torch.equal(ra.topk_val, rb.topk_val), s
    ba, bb = A.ahpp_query_batch(a, srcs, 1e-7, k=40), A.ahpp_query_batch(b, srcs, 1e-7, k=40)
    assert torch.equal(ba.pi, bb.pi) and torch.equal(ba.topk_idx, bb.topk_idx)
    # The walks draw against prefix sums of the raw weights, which scale
    # exactly too: the same seed stops every walk at the same node.
    ma = A.ahpp_query_mc(a, int(srcs[0]), 1_000_000, seed=3)
    mb = A.ahpp_query_mc(b, int(srcs[0]), 1_000_000, seed=3)
    assert torch.equal(ma["pi"], mb["pi"])
    a.free()
    b.free()


def test_repeated_pairs_equal_summed_weight(env):
    torch, A = env
    g = synth.make_custom(5000, 2000, 45000, 200, 6, seed=613, unit_weights=False)
    rng = np.random.default_rng(614)
    se, sa = rng.random(g.edge_u.size) < 0.4, rng.random(g.assoc_u.size) < 0.4
    ew = np.where(se, g.edge_w / 2, g.edge_w).astype(np.float32)
    aw = np.where(sa, g.assoc_w / 2, g.assoc_w).astype(np.float32)
    h = _ns(g, edge_u=np.concatenate([g.edge_u, g.edge_u[se]]), edge_v=np.concatenate([g.edge_v, g.edge_v[se]]),
            edge_w=np.concatenate([ew, ew[se]]),
            assoc_u=np.concatenate([g.assoc_u, g.assoc_u[sa]]), assoc_a=np.concatenate([g.assoc_a, g.assoc_a[sa]]),
            assoc_w=np.concatenate([aw, aw[sa]]))
    _say("split pairs", int(se.sum()), int(sa.sum()))
    og = O.OracleGraph.from_graph(g)
    dh = A.load_graph(h)
    assert dh.lam == pytest.approx(og.lambda_thm3(T=dh.info["lambda_iters"]) * (1 + 1e-4), rel=2e-5)
    srcs = synth.degree_queries(g, 4, 615)
    batch = A.ahpp_query_batch(dh, srcs, 1e-7, k=30)
    for q, s in enumerate(srcs.tolist()):
        exact, _ = og.power_series(s)
        res = A.ahpp_query(dh, s, 1e-7, k=30, want_resid=True)
        chk = O.check_query(exact, res.pi.cpu().numpy().astype(np.float64), 1e-7, tol=TOL,
                            resid=res.resid.cpu().numpy().astype(np.float64), k=30, source=s,
                            topk_ids=res.topk_idx[: int(res.topk_n.item())].cpu().numpy())
        assert chk.ok, (s, chk.detail)
        chk = O.check_query(exact, batch.pi[q].cpu().numpy().astype(np.float64), 1e-7, tol=TOL, k=30, source=s,
                            topk_ids=batch.topk_idx[q, : int(batch.topk_n[q].item())].cpu().numpy())
        assert chk.ok, (s, "batched", chk.detail)
    # Walks on the split graph: every node within six standard deviations of
    # the original graph's exact row (stop counts are binomial, Lemma 1).
    s = int(srcs[0])
    exact, _ = og.power_series(s)
    n = 4_000_000
    est = A.ahpp_query_mc(dh, s, n, seed=9)["pi"].cpu().numpy().astype(np.float64)
    sd = np.sqrt(np.clip(exact * (1.0 - exact), 0.0, None) / n)
    assert (np.abs(est - exact) <= 6.0 * sd + 3.0 / n).all()
    og.close()
    dh.free()


def test_disjoint_union_keeps_walks_apart(env):
    torch, A = env
    a = synth.make_custom(4000, 1500, 30000, 150, 5, seed=616, unit_weights=False)
    b = synth.make_custom(2500, 1100, 20000, 90, 4, seed=617, unit_weights=False)
    u = _ns(a, n_u=a.n_u + b.n_u, n_v=a.n_v + b.n_v, n_attr=a.n_attr + b.n_attr,
            edge_u=np.concatenate([a.edge_u, b.edge_u + a.n_u]).astype(np.int32),
            edge_v=np.concatenate([a.edge_v, b.edge_v + a.n_v]).astype(np.int32),
            edge_w=np.concatenate([a.edge_w, b.edge_w]),
            assoc_u=np.concatenate([a.assoc_u, b.assoc_u + a.n_u]).astype(np.int32),
            assoc_a=np.concatenate([a.assoc_a, b.assoc_a + a.n_attr]).astype(np.int32),
            assoc_w=np.concatenate([a.assoc_w, b.assoc_w]))
    _say("disjoint union", u.n_u, u.n_v, u.n_attr)
    ou = O.OracleGraph.from_graph(u)
    du = A.load_graph(u)
    srcs = np.concatenate([synth.degree_queries(a, 3, 618), synth.degree_queries(b, 3, 619) + a.n_u]).astype(np.int32)
    batch = A.ahpp_query_batch(du, srcs, 1e-7, k=25)
    for q, s in enumerate(srcs.tolist()):
        own = np.zeros(u.n_u, bool)
        if s < a.n_u:
            own[: a.n_u] = True
        else:
            own[a.n_u:] = True
        res = A.ahpp_query(du, s, 1e-7, k=25, want_resid=True)
        pi, r = res.pi.cpu().numpy(), res.resid.cpu().numpy()
        assert np.all(pi[~own] == 0) and np.all(r[~own] == 0), s
        assert np.all(batch.pi[q].cpu().numpy()[~own] == 0), (s, "batched")
        ids = res.topk_idx[: int(res.topk_n.item())].cpu().numpy()
        assert own[ids].all(), s
        exact, _ = ou.power_series(s)
        chk = O.check_query(exact, pi.astype(np.float64), 1e-7, tol=TOL, resid=r.astype(np.float64), k=25,
                            source=s, topk_ids=ids)
        assert chk.ok, (s, chk.detail)
        # Exp-2's schedules and the walks stay in the component too.
        for sch in (1, 3):
            rs = A.ahpp_query_schedule(du, s, 1e-7, sch, want_resid=True)
            assert np.all(rs.pi.cpu().numpy()[~own] == 0) and np.all(rs.resid.cpu().numpy()[~own] == 0), (s, sch)
        mc = A.ahpp_query_mc(du, s, 500_000, seed=q)["pi"].cpu().numpy()
        assert np.all(mc[~own] == 0) and mc[own].sum() > 0.99, s
    ou.close()
    du.free()
