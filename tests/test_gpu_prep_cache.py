"""The lambda cache of ahpp_graph_load (cache_dir) on the device.

A first load computes lambda (Theorem 3, Eq. 6) and files it under the key
of the inputs; a second load of the same inputs reads it instead of running
the sweeps.  The key the device computes over the uploaded COO equals the
host's ahpp_graph_key, and the cached load answers queries bit for bit as
the fresh one.  Changed inputs get a new key; a damaged entry is ignored.
"""

import os

import numpy as np
import pytest

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


def test_cached_load_equals_fresh_load(env, tmp_path):
    ahpp, torch = env
    g = synth.make_custom(6000, 2500, 60000, 300, 8, seed=515, unit_weights=False)
    d = str(tmp_path)
    _say("fresh load with cache dir")
    a = ahpp.load_graph(g, cache_dir=d)
    ia = ahpp.ahpp_graph_info(a)
    assert ia["lambda_cached"] == 2
    assert ia["key"] == ahpp.ahpp_graph_key(g)
    files = [f for f in os.listdir(d) if f.endswith(".lambda")]
    assert files == ["ahpp-%016x%016x.lambda" % ia["key"]]
    _say("cached load")
    b = ahpp.load_graph(g, cache_dir=d)
    ib = ahpp.ahpp_graph_info(b)
    assert ib["lambda_cached"] == 1 and ib["key"] == ia["key"]
    assert ib["lam"] == ia["lam"] and ib["lambda_iters"] == ia["lambda_iters"]
    srcs = synth.degree_queries(g, 300, 2041)
    ra = ahpp.ahpp_query(a, int(srcs[0]), 1e-6, k=20, want_resid=True)
    rb = ahpp.ahpp_query(b, int(srcs[0]), 1e-6, k=20, want_resid=True)
    ba = ahpp.ahpp_query_batch(a, srcs, 1e-6, k=20)
    bb = ahpp.ahpp_query_batch(b, srcs, 1e-6, k=20)
    torch.cuda.synchronize()
    for x, y in ((ra.pi, rb.pi), (ra.resid, rb.resid), (ba.pi, bb.pi), (ba.topk_val, bb.topk_val)):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))
    assert torch.equal(ba.topk_idx, bb.topk_idx)
    a.free()
    b.free()
    # Another alpha is another key and another entry; a damaged entry is recomputed.
    c = ahpp.load_graph(g, alpha=0.2, cache_dir=d)
    ic = ahpp.ahpp_graph_info(c)
    assert ic["key"] != ia["key"] and ic["lambda_cached"] == 2
    c.free()
    path = os.path.join(d, "ahpp-%016x%016x.lambda" % ia["key"])
    with open(path, "r+b") as f:
        f.seek(8)
        f.write(b"\0" * 8)
    e = ahpp.load_graph(g, cache_dir=d)
    ie = ahpp.ahpp_graph_info(e)
    assert ie["lambda_cached"] == 2 and ie["lam"] == ia["lam"]
    e.free()
    # No cache dir: nothing read or written.
    f0 = ahpp.load_graph(g)
    assert ahpp.ahpp_graph_info(f0)["lambda_cached"] == 0
    f0.free()
