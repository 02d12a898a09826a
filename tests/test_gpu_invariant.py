"""Lemma 2 on the device after every round count.

A query stopped by its round cap hands back its reserves and U residues; for
any state the push can reach, pi(s, t) = reserve(t) + sum_i r(i) pi(i, t)
holds (Lemma 2), with pi from a dense solve.  Checked for the four push
schedules, at caps from one round up to convergence, on a unit-weight and a
weighted graph.  The float32 state may differ from the oracle's in which
residues cross a threshold, so the invariant, not the oracle's trace, is the
reference here.
"""

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth

pytestmark = pytest.mark.gpu

TOL = 2e-6


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


@pytest.fixture(scope="module")
def weighted():
    g = synth.make_custom(1500, 700, 12000, 60, 4, seed=621, unit_weights=False)
    return g, O.exact_dense(g)


@pytest.mark.parametrize("which", ["unit", "weighted"])
@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
def test_lemma2_after_each_cap(env, tiny_graph, tiny_Pi, weighted, which, schedule):
    torch, A = env
    g, Pi = (tiny_graph, tiny_Pi) if which == "unit" else weighted
    dg = A.load_graph(g)
    for s in synth.degree_queries(g, 2, 622).tolist():
        full = A.ahpp_query_schedule(dg, s, 1e-6, schedule, want_resid=True)
        n_full = None
        for n in (1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 1000):
            _say(which, "schedule", schedule, "source", s, "cap", n)
            res = A.ahpp_query_schedule(dg, s, 1e-6, schedule, max_iters=n, want_resid=True,
                                        allow_not_converged=True)
            pi = res.pi.cpu().numpy().astype(np.float64)
            r = res.resid.cpu().numpy().astype(np.float64)
            assert pi.min() >= 0 and r.min() >= 0
            err = np.abs(pi + r @ Pi - Pi[s]).max()
            assert err <= TOL, (which, schedule, s, n, err)
            if res.status == 0:
                # Converged within the cap: the same answer as without one.
                assert torch.equal(res.pi, full.pi) and torch.equal(res.resid, full.resid), (schedule, s, n)
                n_full = n
                break
        assert n_full is not None, (which, schedule, s, "did not converge within 1000 rounds")
    dg.free()
