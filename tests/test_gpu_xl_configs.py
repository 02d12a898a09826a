"""Full-size runs of the two large workload shapes.

* Serving on the 5M / 2M / 100M graph (50k attributes x 30, Zipf 2.0
  degrees): Poisson arrivals, eps drawn from {1e-5, 1e-6, 1e-7, 1e-8}, k = 50,
  512 slots.  Every result is checked for properties that hold at any size;
  two sampled queries are checked in full against the oracle's exact series
  and against the same query run alone.
* A batch of 256 hub sources on the 20M / 10M / 500M graph (50k attributes x
  100, Zipf 1.3 popularity) at eps = 1e-7, k = 100.  Each of the 256 results
  is checked for properties that hold at any size: no negative score, mass
  conservation (sum of scores + sum of residues = 1, Lemma 2 summed over U),
  the stop rule (max residue <= eps / lambda), top-k equal to a host sort of
  the returned vector, and agreement with the independent single-query path
  for two sources.  The first source is checked in full against the oracle's
  exact series (Theorem 2's bound and the top-k band); its FP64 adjacency
  (about 60 GB of host memory) is built and the series run on a host thread
  while the device works.
"""

import threading
import time

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6
EPS_SET = (1e-5, 1e-6, 1e-7, 1e-8)


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    assert synth.native_lib() is not None, "libsynth.so must be built for the large graphs"
    return ahpp, torch


def _host_topk(pi, k, source):
    x = pi.astype(np.float64).copy()
    x[source] = -np.inf
    order = np.lexsort((np.arange(x.size), -x))
    top = order[:k]
    return top[x[top] > 0]


@pytest.mark.timeout(1100)
def test_serving_on_the_5m_graph(env):
    ahpp, torch = env
    t0 = time.time()
    g = synth.make_graph("serve5m")
    _say(f"generated serve5m in {time.time() - t0:.1f} s: m_e={g.m_e} m_a={g.m_a}")
    dg = ahpp.load_graph(g)
    info = ahpp.ahpp_graph_info(dg)
    _say("loaded; lambda", dg.lam, "dangling", info["dangling_u"])
    assert info["dangling_u"] == 0
    from paper_2512_11606_amd import serve
    n = 160
    srcs = synth.degree_queries(g, n, 2003)
    pick = (synth.CounterRNG(2003, "serve_eps").uniform(n) * 4).astype(int)
    eps = [EPS_SET[min(i, 3)] for i in pick]
    srv = ahpp.Server(dg, k=50, max_slots=512, keep_pi=True)
    summary, res = serve.run(srv, srcs, eps, rate_qps=40.0, rounds_per_step=4, want_pi=True, max_wall_s=600.0)
    srv.close()
    _say("serving summary", summary)
    assert summary["completed"] == n
    for t, r in res.items():
        st = r["stats"]
        pi = r["pi"]
        assert st["converged"] == 1, t
        assert st["max_residual"] <= eps[t] / dg.lam * (1 + 1e-6), t
        assert float(pi.min().item()) >= 0.0, t
        assert abs(float(pi.sum(dtype=torch.float64).item()) + st["sum_residual"] - 1.0) < 1e-5, t
    # Two sampled queries: the busiest source and the first one, in full.
    deg = g.u_degree_counts()
    hub_t = int(np.argmax(deg[srcs]))
    sample = [hub_t, 0] if hub_t != 0 else [0, 1]
    og = O.OracleGraph.from_graph(g)
    for t in sample:
        s, e = int(srcs[t]), float(eps[t])
        t1 = time.time()
        exact, tail = og.power_series(s)
        _say(f"oracle series for source {s} (eps {e:g}) in {time.time() - t1:.1f} s, tail {tail:.1e}")
        r = res[t]
        mix = r["pi"].cpu().numpy().astype(np.float64)
        chk = O.check_query(exact, mix, e, tol=TOL, k=50, source=s, topk_ids=r["topk_idx"])
        _say("check", t, chk.ok, f"max |err| {chk.max_abs_err:.3e}")
        assert chk.ok, (t, s, e, chk.detail)
        alone = ahpp.ahpp_query(dg, s, e, k=50)
        assert np.abs(alone.pi.cpu().numpy().astype(np.float64) - mix).max() <= e + TOL
    og.close()
    dg.free()


@pytest.mark.timeout(1100)
def test_hub_batch_on_the_20m_graph(env):
    ahpp, torch = env
    t0 = time.time()
    g = synth.make_graph("large20m")
    _say(f"generated large20m in {time.time() - t0:.1f} s: m_e={g.m_e} m_a={g.m_a}")
    t0 = time.time()
    dg = ahpp.load_graph(g)
    info = ahpp.ahpp_graph_info(dg)
    _say(f"loaded in {time.time() - t0:.1f} s; lambda {dg.lam}; build {info['load_ms']:.0f} ms, "
         f"lambda {info['lambda_ms']:.0f} ms; device bytes {info['device_bytes']}")
    assert info["dangling_u"] == 0
    eps, k = 1e-7, 100
    srcs = synth.hub_queries(g, 256, 2004)
    # The oracle's exact row of the first source, on a host thread (its C
    # calls release the GIL) while the device runs the batch.
    box = {}

    def oracle_job():
        try:
            t = time.time()
            og = O.OracleGraph.from_graph(g)
            box["build_s"] = time.time() - t
            _say(f"oracle adjacency built in {box['build_s']:.1f} s")
            t = time.time()

            def report(done, total):
                if done % 32 == 0 or done == total:
                    _say(f"oracle series: {done} of {total} terms, {time.time() - t:.1f} s")

            box["exact"], box["tail"] = og.power_series(int(srcs[0]), progress=report)
            box["series_s"] = time.time() - t
            og.close()
        except BaseException as e:  # noqa: BLE001 - re-raised below
            box["error"] = e

    job = threading.Thread(target=oracle_job, daemon=True)
    job.start()
    t0 = time.time()
    res = ahpp.ahpp_query_batch(dg, srcs, eps, k=k)
    torch.cuda.synchronize()
    dt = time.time() - t0
    _say(f"batch of 256 hub queries: {dt:.1f} s, {256 / dt:.2f} queries/s, rounds {res.stats[0]['iters']}")
    pi = res.pi
    mins = pi.min(dim=1).values.cpu().numpy()
    sums = pi.sum(dim=1, dtype=torch.float64).cpu().numpy()
    for q in range(srcs.size):
        st = res.stats[q]
        assert st["converged"] == 1, q
        assert st["max_residual"] <= eps / dg.lam * (1 + 1e-6), q
        assert mins[q] >= 0.0, q
        assert abs(sums[q] + st["sum_residual"] - 1.0) < 1e-5, (q, sums[q], st["sum_residual"])
    for q in (0, 97, 255):
        host = pi[q].cpu().numpy()
        want = _host_topk(host, k, int(srcs[q]))
        n_q = int(res.topk_n[q].item())
        got = res.topk_idx[q, :n_q].cpu().numpy()
        assert np.array_equal(got, want), q
    for q in (0, 255):
        alone = ahpp.ahpp_query(dg, int(srcs[q]), eps, k=k)
        d = np.abs(alone.pi.cpu().numpy().astype(np.float64) - pi[q].cpu().numpy().astype(np.float64)).max()
        _say(f"batch vs alone, query {q}: max |diff| {d:.3e}")
        assert d <= eps + TOL
    row0 = pi[0].cpu().numpy().astype(np.float64)
    top0 = res.topk_idx[0, : int(res.topk_n[0].item())].cpu().numpy()
    del pi, res
    dg.free()
    _say("waiting for the oracle's exact series")
    job.join()
    if "error" in box:
        raise box["error"]
    s = int(srcs[0])
    _say(f"oracle: adjacency {box['build_s']:.1f} s, series for source {s} {box['series_s']:.1f} s, "
         f"tail {box['tail']:.1e}")
    assert box["tail"] < 1e-11
    chk = O.check_query(box["exact"], row0, eps, tol=TOL, k=k, source=s, topk_ids=top0)
    _say("oracle check", chk.ok, f"max |err| {chk.max_abs_err:.3e} = {chk.max_abs_err / eps:.3f} eps")
    assert chk.ok, chk.detail


@pytest.mark.timeout(900)
def test_amazon_shaped_graph(env):
    """The graph of the paper's Amazon sizes (2.3M/8.0M/22.5M, 800 attributes
    x 10) at eps = 1e-6, the setting of its scalability figure: two plain
    queries in full against the oracle's exact series, and a batch of 256
    whose results agree with the plain path."""
    ahpp, torch = env
    g = synth.make_graph("amazon")
    dg = ahpp.load_graph(g)
    _say("loaded amazon-shaped graph; lambda", dg.lam)
    eps = 1e-6
    srcs = synth.degree_queries(g, 256, 2005)
    og = O.OracleGraph.from_graph(g)
    plain = {}
    for q in (0, 1):
        s = int(srcs[q])
        t0 = time.time()
        r = ahpp.ahpp_query(dg, s, eps, k=50, want_resid=True)
        torch.cuda.synchronize()
        _say(f"plain query {s}: {(time.time() - t0) * 1e3:.1f} ms, {r.stats[0]['iters']} rounds")
        exact, tail = og.power_series(s)
        pi = r.pi.cpu().numpy().astype(np.float64)
        chk = O.check_query(exact, pi, eps, tol=TOL, resid=r.resid.cpu().numpy(), k=50, source=s,
                            topk_ids=r.topk_idx[: int(r.topk_n.item())].cpu().numpy())
        _say("check", q, chk.ok, f"max |err| {chk.max_abs_err:.3e}")
        assert chk.ok, chk.detail
        plain[q] = pi
    og.close()
    res = ahpp.ahpp_query_batch(dg, srcs, eps, k=50)
    sums = res.pi.sum(dim=1, dtype=torch.float64).cpu().numpy()
    for q in range(srcs.size):
        st = res.stats[q]
        assert st["converged"] == 1 and st["max_residual"] <= eps / dg.lam * (1 + 1e-6), q
        assert abs(sums[q] + st["sum_residual"] - 1.0) < 1e-5, q
    for q in (0, 1):
        assert np.abs(res.pi[q].cpu().numpy().astype(np.float64) - plain[q]).max() <= eps + TOL
    dg.free()
