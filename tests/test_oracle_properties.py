"""Metamorphic properties of the CPU oracle on generated tiny graphs.

Each property follows from the definitions alone, independent of how the
oracle sums:

* Eq. 1 and Eq. 2 divide every weight by a sum of weights of the same kind,
  so multiplying all edge weights by one constant and all attribute weights by
  another leaves P, and so every AHPP score, unchanged.  With power-of-two
  constants every rounding step scales with the weights, so the scores stay
  equal bit for bit.
* Both equations are linear in each weight, so a pair listed twice with
  weights a and b is the pair listed once with weight a + b.
* Renaming the nodes of U, V and the attribute set permutes the scores.
* A walk never leaves its connected component, so a source in one of two
  disjoint graphs scores exactly zero on the other, and its scores on its own
  graph are those of that graph alone; the residue push of Algorithm 4
  touches nothing outside the component either.

A slip such as a missing normaliser, a weight used where its normalised value
belongs, or an index taken from the wrong side breaks one of these.
"""

import types

import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle as O

WEIGHTS = [0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 5.0]
SETTINGS = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])


def _graph(n_u, n_v, n_attr, eu, ev, ew, au, aa, aw):
    return types.SimpleNamespace(
        n_u=n_u, n_v=n_v, n_attr=n_attr,
        edge_u=np.asarray(eu, np.int32), edge_v=np.asarray(ev, np.int32), edge_w=np.asarray(ew, np.float32),
        assoc_u=np.asarray(au, np.int32), assoc_a=np.asarray(aa, np.int32), assoc_w=np.asarray(aw, np.float32))


@st.composite
def tiny_graphs(draw):
    n_u = draw(st.integers(2, 8))
    n_v = draw(st.integers(1, 6))
    n_attr = draw(st.integers(1, 4))
    m_e = draw(st.integers(1, 3 * n_u))
    m_a = draw(st.integers(0, 2 * n_u))
    eu = draw(st.lists(st.integers(0, n_u - 1), min_size=m_e, max_size=m_e))
    ev = draw(st.lists(st.integers(0, n_v - 1), min_size=m_e, max_size=m_e))
    ew = draw(st.lists(st.sampled_from(WEIGHTS), min_size=m_e, max_size=m_e))
    au = draw(st.lists(st.integers(0, n_u - 1), min_size=m_a, max_size=m_a))
    aa = draw(st.lists(st.integers(0, n_attr - 1), min_size=m_a, max_size=m_a))
    aw = draw(st.lists(st.sampled_from(WEIGHTS), min_size=m_a, max_size=m_a))
    source = draw(st.integers(0, n_u - 1))
    return _graph(n_u, n_v, n_attr, eu, ev, ew, au, aa, aw), source


def _series(g, source, beta=O.BETA):
    pi, _ = O.OracleGraph.from_graph(g).power_series(source, beta=beta)
    return pi


@SETTINGS
@given(tiny_graphs(), st.sampled_from([0.25, 2.0, 8.0]), st.sampled_from([0.5, 4.0, 16.0]))
def test_power_of_two_weight_scaling_is_exact(gs, ce, ca):
    g, s = gs
    h = _graph(g.n_u, g.n_v, g.n_attr, g.edge_u, g.edge_v, g.edge_w * ce, g.assoc_u, g.assoc_a, g.assoc_w * ca)
    assert np.array_equal(_series(g, s), _series(h, s))


@SETTINGS
@given(tiny_graphs(), st.sampled_from([3.0, 0.7]), st.sampled_from([1.3, 11.0]))
def test_weight_scaling_leaves_scores(gs, ce, ca):
    g, s = gs
    h = _graph(g.n_u, g.n_v, g.n_attr, g.edge_u, g.edge_v, g.edge_w * ce, g.assoc_u, g.assoc_a, g.assoc_w * ca)
    # float32 products round, so the weights agree to 2^-24 relative.
    np.testing.assert_allclose(_series(h, s), _series(g, s), rtol=1e-6, atol=1e-12)


@SETTINGS
@given(tiny_graphs(), st.data())
def test_repeated_pairs_equal_summed_weight(gs, data):
    g, s = gs
    split_e = data.draw(st.lists(st.booleans(), min_size=g.edge_u.size, max_size=g.edge_u.size))
    split_a = data.draw(st.lists(st.booleans(), min_size=g.assoc_u.size, max_size=g.assoc_u.size))
    se, sa = np.asarray(split_e, bool), np.asarray(split_a, bool)
    # A split pair becomes two entries of half the weight (exact in float32),
    # the second one appended at the end of the list.
    ew = np.where(se, g.edge_w / 2, g.edge_w)
    aw = np.where(sa, g.assoc_w / 2, g.assoc_w)
    h = _graph(g.n_u, g.n_v, g.n_attr,
               np.concatenate([g.edge_u, g.edge_u[se]]), np.concatenate([g.edge_v, g.edge_v[se]]),
               np.concatenate([ew, ew[se]]),
               np.concatenate([g.assoc_u, g.assoc_u[sa]]), np.concatenate([g.assoc_a, g.assoc_a[sa]]),
               np.concatenate([aw, aw[sa]]))
    np.testing.assert_allclose(_series(h, s), _series(g, s), rtol=1e-12, atol=1e-15)


@SETTINGS
@given(tiny_graphs(), st.integers(0, 2 ** 32 - 1))
def test_renaming_nodes_permutes_scores(gs, seed):
    g, s = gs
    rng = np.random.default_rng(seed)
    pu, pv, pa = rng.permutation(g.n_u), rng.permutation(g.n_v), rng.permutation(g.n_attr)
    order_e, order_a = rng.permutation(g.edge_u.size), rng.permutation(g.assoc_u.size)
    h = _graph(g.n_u, g.n_v, g.n_attr,
               pu[g.edge_u][order_e], pv[g.edge_v][order_e], g.edge_w[order_e],
               pu[g.assoc_u][order_a], pa[g.assoc_a][order_a], g.assoc_w[order_a])
    got = _series(h, int(pu[s]))
    np.testing.assert_allclose(got[pu], _series(g, s), rtol=1e-12, atol=1e-15)


def _union(a, b):
    return _graph(a.n_u + b.n_u, a.n_v + b.n_v, a.n_attr + b.n_attr,
                  np.concatenate([a.edge_u, b.edge_u + a.n_u]), np.concatenate([a.edge_v, b.edge_v + a.n_v]),
                  np.concatenate([a.edge_w, b.edge_w]),
                  np.concatenate([a.assoc_u, b.assoc_u + a.n_u]), np.concatenate([a.assoc_a, b.assoc_a + a.n_attr]),
                  np.concatenate([a.assoc_w, b.assoc_w]))


@SETTINGS
@given(tiny_graphs(), tiny_graphs(), st.booleans())
def test_disjoint_union_keeps_walks_apart(ga, gb, second):
    (a, sa), (b, sb) = ga, gb
    u = _union(a, b)
    own, n_own = (b, b.n_u) if second else (a, a.n_u)
    src = (a.n_u + sb) if second else sa
    lo = a.n_u if second else 0
    pi = _series(u, src)
    mask = np.zeros(u.n_u, bool)
    mask[lo: lo + n_own] = True
    assert np.all(pi[~mask] == 0.0)
    np.testing.assert_allclose(pi[mask], _series(own, sb if second else sa), rtol=1e-12, atol=1e-15)
    og = O.OracleGraph.from_graph(u)
    res, r, _, ok = og.asrp(src, 1e-6, og.lambda_thm3())
    assert ok and np.all(res[~mask] == 0.0) and np.all(r[~mask] == 0.0)


def test_scaling_catches_a_dropped_normaliser():
    """The slip of Eq. 1 with d(v) left out is not scale-free, so the scaling
    property above would fail on it, while the true form passes."""
    def slipped(g):
        W = np.zeros((g.n_u, g.n_v))
        np.add.at(W, (g.edge_u, g.edge_v), g.edge_w.astype(np.float64))
        return (W / W.sum(1, keepdims=True)) @ W.T

    g = _graph(3, 2, 1, [0, 1, 1, 2], [0, 0, 1, 1], [1.0, 2.0, 1.0, 3.0], [0, 2], [0, 0], [1.0, 1.0])
    h = _graph(3, 2, 1, g.edge_u, g.edge_v, g.edge_w * 2, g.assoc_u, g.assoc_a, g.assoc_w)
    assert np.array_equal(O.dense_PS(g), O.dense_PS(h))
    assert np.abs(slipped(h) - slipped(g)).max() > 0.5
