"""The push schedules of Exp-2 on the GPU (ASRP, APP, APP(S), APP(E)) against
the oracle: each result meets the eps bound against the exact row, APP(E)
stops under eps / lambda and APP / APP(S) under their per-node thresholds,
and the round counts and phase switches follow the oracle's double-precision
run of the same schedule (within a few rounds: float32 threshold tests can
flip a node near its threshold)."""

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6
NAMES = {0: "ASRP", 1: "APP", 2: "APP(S)", 3: "APP(E)"}


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11606_amd import ahpp
    g = synth.make_custom(5000, 2000, 40000, 200, 6, seed=1212, unit_weights=False)
    dg = ahpp.load_graph(g)
    yield g, dg, O.OracleGraph.from_graph(g), ahpp, torch
    dg.free()


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
@pytest.mark.parametrize("eps", [1e-5, 1e-7])
def test_schedule_meets_bound(env, schedule, eps):
    g, dg, og, ahpp, torch = env
    deg = (np.bincount(g.edge_u, minlength=g.n_u) + np.bincount(g.assoc_u, minlength=g.n_u)).astype(np.float64)
    thr = eps / (g.m_e + g.m_a) * deg
    for s in synth.mixed_batch_queries(g, 2, 41).tolist():
        res = ahpp.ahpp_query_schedule(dg, s, eps, schedule, k=25, want_resid=True)
        st = res.stats[0]
        exact, _ = og.power_series(s)
        pi = res.pi.cpu().numpy().astype(np.float64)
        r = res.resid.cpu().numpy().astype(np.float64)
        chk = O.check_query(exact, pi, eps, tol=TOL, resid=r, k=25, source=s,
                            topk_ids=res.topk_idx[: int(res.topk_n.item())].cpu().numpy())
        _, _, ost, ok = og.push_schedule(s, eps, dg.lam, schedule)
        _say(NAMES[schedule], eps, s, "gpu rounds", st["iters"], "oracle", ost.iterations, "switch", st["sync_switch_iter"],
             ost.switch_iteration, "max |err|", f"{chk.max_abs_err:.2e}")
        assert chk.ok, chk.detail
        assert st["converged"] == 1 and ok
        if schedule in (0, 3):
            assert r.max() <= eps / dg.lam * (1 + 1e-6)
        else:
            assert (r <= thr * (1 + 1e-5) + 1e-30).all()
            assert st["max_residual"] <= 1.0
        assert abs(st["iters"] - ost.iterations) <= 3
        if schedule in (1, 3):
            assert st["sync_switch_iter"] == -1


def test_asrp_schedule_equals_plain_query(env):
    g, dg, og, ahpp, torch = env
    s = int(synth.degree_queries(g, 1, 5)[0])
    a = ahpp.ahpp_query(dg, s, 1e-7)
    b = ahpp.ahpp_query_schedule(dg, s, 1e-7, 0)
    assert torch.equal(a.pi, b.pi) and a.stats[0]["iters"] == b.stats[0]["iters"]


def test_bad_schedule_is_rejected(env):
    g, dg, og, ahpp, torch = env
    with pytest.raises(ahpp.AhppError) as e:
        ahpp.ahpp_query_schedule(dg, 0, 1e-6, 4)
    assert e.value.status == ahpp.ERR_INVALID_ARG


def test_app_agrees_with_forward_push(env):
    """Algorithm 2 (FP) pushes one node at a time; run level-synchronously on
    the device it is APP's round.  Both stop with every residue under
    r_max (|N(u)| + |A(u)|) and under-estimate the exact row by at most eps,
    so the device's APP and the oracle's node-at-a-time FP agree within eps."""
    _, _, _, ahpp, torch = env
    # A smaller graph: FP's two-hop pushes cost the oracle about a second here.
    g = synth.make_custom(1500, 600, 12000, 60, 6, seed=1213, unit_weights=False)
    og = O.OracleGraph.from_graph(g)
    dg = ahpp.load_graph(g)
    eps = 1e-6
    s = int(synth.degree_queries(g, 1, 77)[0])
    fp, _, fst, ok = og.forward_push(s, eps / (g.m_e + g.m_a))
    assert ok
    res = ahpp.ahpp_query_schedule(dg, s, eps, 1)
    dg.free()
    d = np.abs(res.pi.cpu().numpy().astype(np.float64) - fp).max()
    _say("APP vs FP", s, "pushes", fst.iterations, f"max |diff| {d:.2e}")
    assert d <= eps + TOL
