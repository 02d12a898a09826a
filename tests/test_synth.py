"""Seeded input generators: determinism and the structure the recipe promises."""

import dataclasses

import numpy as np
import pytest

from paper_2512_11606_amd import synth


def test_tiny_is_deterministic_and_well_formed():
    a = synth.make_graph("tiny")
    b = synth.make_graph("tiny")
    for f in ("edge_u", "edge_v", "edge_w", "assoc_u", "assoc_a", "assoc_w"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    keys = a.edge_u.astype(np.int64) * a.n_v + a.edge_v
    assert np.unique(keys).size == keys.size                     # distinct pairs
    assert a.m_e >= 20_000
    assert np.bincount(a.edge_u, minlength=a.n_u).min() >= 1     # no edgeless U node
    cnt = np.bincount(a.assoc_u, minlength=a.n_u)
    assert (cnt == 5).all()                                      # c distinct attributes each
    ak = a.assoc_u.astype(np.int64) * a.n_attr + a.assoc_a
    assert np.unique(ak).size == ak.size
    assert (a.edge_w == 1).all() and (a.assoc_w == 1).all()


def test_weighted_ranges_and_power_law():
    g = synth.make_custom(3000, 1500, 30000, 200, 6, seed=77)
    assert g.edge_w.min() >= 0.5 and g.edge_w.max() <= 1.0
    assert g.assoc_w.min() > 0 and g.assoc_w.max() <= 1.0
    deg = np.bincount(g.edge_u, minlength=g.n_u)
    # heavy tail: the largest degree is far above the mean
    assert deg.max() > 10 * deg.mean()
    pop = np.bincount(g.assoc_a, minlength=g.n_attr)
    assert pop.max() > 0.5 * g.n_u                               # Zipf(1.5) head attribute


def test_query_sets():
    g = synth.make_graph("tiny")
    q = synth.mixed_batch_queries(g, 64, 2002)
    assert np.unique(q).size == 64 and q.min() >= 0 and q.max() < g.n_u
    deg = g.u_degree_counts()
    top = set(np.argsort(-deg, kind="stable")[: g.n_u // 100].tolist())
    assert sum(int(x) in top for x in q[:20]) == 20
    d = synth.degree_queries(g, 1000, 5)
    assert deg[d].mean() > deg.mean()                            # degree-biased
    u = synth.uniform_queries(g, 10, 1)
    assert np.array_equal(u, synth.uniform_queries(g, 10, 1))


def _native_lib():
    import os
    from paper_2512_11606_amd import build
    if not os.path.exists(build.SYNTH_LIB):
        build.build_synth()
    lib = synth.native_lib()
    assert lib is not None
    return lib


FIELDS = ("edge_u", "edge_v", "edge_w", "assoc_u", "assoc_a", "assoc_w")


def test_native_generator_matches_numpy_definition():
    """libsynth.so repeats synth.py's steps: identical arrays, including
    heavy edge rejection (few V nodes), the over-full last round, lonely U
    nodes, and attribute lists that need several rejection rounds."""
    _native_lib()
    cases = [("tiny", None), ((5000, 2000, 40000, 200, 6, 717), {}),
             ((3000, 50, 20000, 30, 25, 9), {}), ((4000, 3000, 4500, 40, 3, 11), {"gamma": 2.6}),
             ((20000, 10000, 300000, 500, 12, 5), {"attr_exponent": 1.3})]
    for args, kw in cases:
        if isinstance(args, str):
            a, b = synth.make_graph(args, native=False), synth.make_graph(args, native=True)
        else:
            a = synth.make_custom(*args, native=False, **kw)
            b = synth.make_custom(*args, native=True, **kw)
        for f in FIELDS:
            x, y = getattr(a, f), getattr(b, f)
            assert x.dtype == y.dtype and np.array_equal(x, y), (args, f)
    # The sparse case really had lonely U nodes to fix and many rejections.
    g = synth.make_custom(4000, 3000, 4500, 40, 3, 11, gamma=2.6, native=True)
    assert np.bincount(g.edge_u, minlength=g.n_u).min() >= 1 and g.m_e > 4500


def test_native_generator_needs_the_library_when_forced(monkeypatch):
    monkeypatch.setattr(synth, "_NATIVE_LIB", None)
    monkeypatch.setattr(synth.os.path, "exists", lambda p: False)
    import pytest
    with pytest.raises(RuntimeError):
        synth.make_graph("tiny", native=True)


@pytest.mark.parametrize("mode", ["nodes", "edges"])
def test_sample_graph_keeps_whole_nodes(mode):
    """Exp-3's sampled graphs: the kept edges and attribute rows are exactly
    those of the kept nodes, ids are renumbered in order, sizes are exact.
    Edge and attribute weights are set to distinct values here, so they
    identify each entry of the original graph."""
    g = synth.make_custom(300, 150, 2500, 30, 3, seed=77, unit_weights=False, native=False)
    g = dataclasses.replace(g, edge_w=(1.0 + np.arange(g.m_e)).astype(np.float32),
                            assoc_w=(1.0 + np.arange(g.m_a)).astype(np.float32))
    s = synth.sample_graph(g, 0.6, mode, seed=5)
    e_of = {float(w): i for i, w in enumerate(g.edge_w)}
    a_of = {float(w): i for i, w in enumerate(g.assoc_w)}
    src = np.array([e_of[float(w)] for w in s.edge_w])
    u_map, v_map = {}, {}
    for new_u, new_v, i in zip(s.edge_u, s.edge_v, src):
        assert u_map.setdefault(int(g.edge_u[i]), int(new_u)) == new_u
        assert v_map.setdefault(int(g.edge_v[i]), int(new_v)) == new_v
    kept_u = np.array(sorted(u_map))
    assert [u_map[u] for u in kept_u] == list(range(kept_u.size)) == list(range(s.n_u))
    assert [v_map[v] for v in sorted(v_map)] == list(range(s.n_v))
    if mode == "nodes":
        assert s.n_u == round(0.6 * g.n_u)  # every U node of the generator has an edge
        want = np.flatnonzero(np.isin(g.edge_u, kept_u))
        assert np.array_equal(np.sort(src), want)
    else:
        assert s.m_e == round(0.6 * g.m_e)
    # Attribute rows: all of the kept U nodes', no others, attribute ids unchanged.
    asrc = np.array([a_of[float(w)] for w in s.assoc_w])
    assert np.array_equal(np.sort(asrc), np.flatnonzero(np.isin(g.assoc_u, kept_u)))
    for new_u, a, i in zip(s.assoc_u, s.assoc_a, asrc):
        assert u_map[int(g.assoc_u[i])] == new_u and g.assoc_a[i] == a
    assert s.n_attr == g.n_attr
