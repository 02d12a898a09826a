"""ahpp_query_noalloc, the allocation-free variant of ahpp_query, against
ahpp_query itself, through the C ABI.

Two graphs in a row, the second smaller, so the second call finds the fixed
device scratch holding the first call's contents: on each, the variant must
equal ahpp_query bit for bit (the same kernels add in the same order) and
meet Theorem 2's bound and the top-k band against the oracle's exact series.
A graph whose query buffers exceed the fixed scratch is refused.
"""

import types

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
    ahpp.load_library()
    return ahpp, torch


def _bits_equal(torch, a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_noalloc_equals_query_on_two_graphs_in_a_row(env):
    ahpp, torch = env
    big = synth.make_custom(20000, 8000, 200000, 500, 8, seed=731, unit_weights=False)
    small = synth.make_graph("tiny")
    cases = [(big, 1e-6, 50), (small, 1e-6, 20)]
    for g, eps, k in cases:
        src = int(synth.degree_queries(g, 1, 2031)[0])
        _say("noalloc vs query", g.n_u, "U nodes, source", src, "eps", eps, "k", k)
        dg = ahpp.load_graph(g)
        try:
            ref = ahpp.ahpp_query(dg, src, eps, k=k, want_resid=True)
            got = ahpp.ahpp_query_noalloc(dg, src, eps, k=k, want_resid=True)
            torch.cuda.synchronize()
            assert _bits_equal(torch, ref.pi, got.pi)
            assert _bits_equal(torch, ref.resid, got.resid)
            n = int(ref.topk_n.item())
            assert n == int(got.topk_n.item()) == k
            assert torch.equal(ref.topk_idx[:n], got.topk_idx[:n])
            assert _bits_equal(torch, ref.topk_val[:n], got.topk_val[:n])
            for f in ("iters", "sync_switch_iter", "converged", "n_push", "max_residual", "sum_residual"):
                assert ref.stats[0][f] == got.stats[0][f], f
            exact, tail = O.OracleGraph.from_graph(g).power_series(src)
            assert tail < 1e-11
            chk = O.check_query(exact, got.pi.cpu().numpy().astype(np.float64), eps, tol=1e-6,
                                resid=got.resid.cpu().numpy().astype(np.float64), k=k, source=src,
                                topk_ids=got.topk_idx[:n].cpu().numpy())
            assert chk.ok, chk.detail
        finally:
            dg.free()


def test_noalloc_refuses_a_graph_above_the_scratch(env):
    ahpp, torch = env
    # 6M U nodes, one edge and one attribute each: the query buffers need
    # about 3 x 24 MB for U vectors alone, above the fixed 64 MiB.
    n_u = 6_000_000
    u = np.arange(n_u, dtype=np.int32)
    g = types.SimpleNamespace(n_u=n_u, n_v=1000, n_attr=10, edge_u=u, edge_v=(u % 1000).astype(np.int32),
                              edge_w=None, assoc_u=u, assoc_a=(u % 10).astype(np.int32), assoc_w=None)
    _say("noalloc refusal, 6M U nodes")
    dg = ahpp.load_graph(g)
    try:
        with pytest.raises(ahpp.AhppError) as e:
            ahpp.ahpp_query_noalloc(dg, 5, 1e-4, k=5)
        assert e.value.status == -1
        assert "scratch" in str(e.value)
    finally:
        dg.free()
