"""The key of a graph's inputs (ahpp_graph_key, host only): it identifies
the inputs a load turns into lambda (Theorem 3, Eq. 6), so it must change
with any id, weight, alpha, beta or round count, and stay put otherwise.
A plain numpy restatement of the documented hash pins the C++ value."""

import numpy as np
import pytest

from paper_2512_11606_amd import synth

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
LANES = (0x9E3779B97F4A7C15, 0xC2B2AE3D27D4EB4F)


@pytest.fixture(scope="module")
def ahpp():
    import os
    from paper_2512_11606_amd import ahpp as A
    if not os.path.exists(A.LIB_PATH):
        from paper_2512_11606_amd import build
        build.build()
    A.load_library()
    return A


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _mix1(z: int) -> int:
    return int(_mix(np.array([z], dtype=np.uint64))[0])


def numpy_key(g, alpha, beta, T):
    """Per lane l: the sum over array k, position i, 32-bit pattern v of
    mix(mix(lane_l + 8 i + k) + v), then the sizes and parameters folded in."""
    arrays = [g.edge_u, g.edge_v, g.edge_w, g.assoc_u, g.assoc_a, g.assoc_w]
    key = []
    for lane in LANES:
        total = 0
        for k, a in enumerate(arrays):
            if a is None or len(a) == 0:
                continue
            v = np.ascontiguousarray(a).view(np.uint32).astype(np.uint64)
            pos = np.arange(v.size, dtype=np.uint64)
            with np.errstate(over="ignore"):
                w = _mix(_mix(np.uint64(lane) + pos * np.uint64(8) + np.uint64(k)) + v)
            total = (total + int(w.sum(dtype=np.uint64))) & 0xFFFFFFFFFFFFFFFF
        a_bits = int(np.float64(alpha).view(np.uint64))
        b_bits = int(np.float64(beta).view(np.uint64))
        flags = (1 if g.edge_w is not None and len(g.edge_w) else 0) | (2 if g.assoc_w is not None and len(g.assoc_w) else 0)
        params = [g.n_u, g.n_v, g.n_attr, len(g.edge_u), len(g.assoc_u), flags, a_bits, b_bits, T, 1]
        h = lane
        for x in params:
            h = _mix1(h ^ (x & 0xFFFFFFFFFFFFFFFF))
        key.append(_mix1(h ^ total))
    return tuple(key)


def test_key_matches_the_documented_hash(ahpp):
    import math
    g = synth.make_custom(300, 120, 2000, 20, 4, seed=77, unit_weights=False)
    T = math.ceil(math.log(0.01 / 300) / math.log(0.85))  # the smallest T with 300 (1 - 0.15)^T <= 0.01
    assert T == 64
    assert ahpp.ahpp_graph_key(g) == numpy_key(g, 0.15, 0.35, T)
    assert ahpp.ahpp_graph_key(g, lambda_iters=50) == numpy_key(g, 0.15, 0.35, 50)
    assert ahpp.ahpp_graph_key(g, lam=2.0) == numpy_key(g, 0.15, 0.35, 0)
    gu = _copy(synth.make_graph("tiny"), edge_w=None, assoc_w=None)  # no weight arrays: every weight 1
    assert ahpp.ahpp_graph_key(gu) == numpy_key(gu, 0.15, 0.35, math.ceil(math.log(0.01 / 2000) / math.log(0.85)))


def _copy(g, **kw):
    import types
    d = {f: getattr(g, f) for f in ("n_u", "n_v", "n_attr", "edge_u", "edge_v", "edge_w", "assoc_u", "assoc_a",
                                   "assoc_w")}
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    d.update(kw)
    return types.SimpleNamespace(**d)


def test_key_changes_with_every_input(ahpp):
    g = synth.make_custom(300, 120, 2000, 20, 4, seed=78, unit_weights=False)
    base = ahpp.ahpp_graph_key(g)
    assert ahpp.ahpp_graph_key(_copy(g)) == base
    assert ahpp.ahpp_graph_key(g, alpha=0.2) != base
    assert ahpp.ahpp_graph_key(g, beta=0.5) != base
    assert ahpp.ahpp_graph_key(g, lambda_iters=40) != base
    seen = {base}
    rng = np.random.default_rng(1)
    for field in ("edge_u", "edge_v", "edge_w", "assoc_u", "assoc_a", "assoc_w"):
        for _ in range(3):
            h = _copy(g)
            a = getattr(h, field)
            i = int(rng.integers(a.size))
            if a.dtype == np.float32:
                a[i] = np.nextafter(a[i], np.float32(2.0))        # one ulp of one weight
            else:
                hi = h.n_u if field.endswith("_u") else (h.n_v if field == "edge_v" else h.n_attr)
                a[i] = (a[i] + 1) % hi
            k = ahpp.ahpp_graph_key(h)
            assert k not in seen, (field, i)
            seen.add(k)
    # swapping two edges is a different input (the key is positional)
    h = _copy(g)
    h.edge_u[[0, 1]] = h.edge_u[[1, 0]]
    h.edge_v[[0, 1]] = h.edge_v[[1, 0]]
    h.edge_w[[0, 1]] = h.edge_w[[1, 0]]
    assert ahpp.ahpp_graph_key(h) != base
    # dropping the weights (all ones) differs from passing weights of one
    ones = _copy(g, edge_w=np.ones(g.edge_u.size, np.float32))
    assert ahpp.ahpp_graph_key(_copy(g, edge_w=None)) != ahpp.ahpp_graph_key(ones)


def test_key_argument_errors(ahpp):
    import ctypes
    d = ahpp.GraphDesc(10, 5, 2, 0, None, None, None, 0, None, None, None, 1.5, 0.35, 0.0, 0, 0)
    key = (ctypes.c_uint64 * 2)()
    lib = ahpp.load_library()
    assert lib.ahpp_graph_key(ctypes.byref(d), key) == ahpp.ERR_INVALID_ARG
    assert b"alpha" in lib.ahpp_last_error()
    d = ahpp.GraphDesc(10, 5, 2, 3, None, None, None, 0, None, None, None, 0.15, 0.35, 0.0, 0, 0)
    assert lib.ahpp_graph_key(ctypes.byref(d), key) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_graph_key(None, key) == ahpp.ERR_INVALID_ARG
