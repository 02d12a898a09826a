"""Seeded synthetic attributed bipartite graphs and query sets.

This module produces inputs only.  It holds none of the AHPP arithmetic: no
normalisers, no transition probabilities, no push.  Both the CPU oracle and
the HIP path read the arrays it returns, so the two sides always see the same
COO lists and the same query nodes.

Graph model (a Chung-Lu bipartite graph with power-law degrees, the shape of
the user-item graphs of the paper's Table 1):

* every node of U and of V draws an i.i.d. degree weight theta ~ Zipf(gamma),
  P(k) proportional to k**-gamma for k >= 1, truncated at the size of the
  opposite side;
* edge endpoints are drawn independently with probability proportional to
  theta on each side (theta is an integer, so each side is an urn holding
  node x theta[x] times); repeated (u, v) pairs are rejected and redrawn until
  there are exactly ``m_e`` distinct pairs; every U node left without an edge
  then gets one edge to a V node drawn proportional to theta_V;
* edge weights are 1.0 (unit graphs) or uniform in [0.5, 1];
* each U node holds ``attrs_per_node`` distinct attributes: the first that
  many distinct ranks of a stream of Zipf(s) draws over ranks 1..n_attr; ranks map to
  attribute ids through a seeded permutation; attribute values are 1.0
  (binary) or 1 - U[0, 1), i.e. in (0, 1].

Randomness is counter based (SplitMix64 of a key derived from seed and stream,
applied to a running counter), so every array is a pure function of the
configuration and does not depend on thread count or call order.

The numpy code below is the definition.  ``synth_native.cpp`` (built into
``libsynth.so``) repeats the same steps multi-threaded, with the same streams,
rejection order and rounding, and is used when built: it makes the 5M and 20M
configurations in seconds instead of hours.  Tests check that both give
identical arrays.
"""

from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


class CounterRNG:
    """Counter-based stream: value i of stream s is mix64(key(seed, s) + i*golden)."""

    def __init__(self, seed: int, stream: str):
        h = hashlib.sha256(f"{seed}:{stream}".encode()).digest()
        self._key = np.uint64(int.from_bytes(h[:8], "little"))
        self._ctr = 0

    @property
    def key(self) -> int:
        return int(self._key)

    def bits(self, n: int) -> np.ndarray:
        idx = np.arange(self._ctr, self._ctr + n, dtype=np.uint64)
        self._ctr += n
        with np.errstate(over="ignore"):
            return _mix64(self._key + idx * _GOLDEN)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) with 53 random bits."""
        return (self.bits(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _zipf_cdf(exponent: float, kmax: int) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-exponent)
    c = np.cumsum(p)
    return c / c[-1]


def _sample_cdf(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Index i with cdf[i-1] <= u < cdf[i] (0-based)."""
    i = np.searchsorted(cdf, u, side="right")
    return np.minimum(i, len(cdf) - 1)


@dataclasses.dataclass
class BipartiteConfig:
    name: str
    n_u: int
    n_v: int
    m_e: int
    gamma_u: float
    gamma_v: float
    n_attr: int
    attrs_per_node: int
    attr_exponent: float
    unit_weights: bool
    seed: int


@dataclasses.dataclass
class AttributedBipartiteGraph:
    """COO lists of one attributed bipartite graph (ids 0-based, int32)."""

    config: BipartiteConfig
    n_u: int
    n_v: int
    n_attr: int
    edge_u: np.ndarray      # int32[m_e]
    edge_v: np.ndarray      # int32[m_e]
    edge_w: np.ndarray      # float32[m_e]
    assoc_u: np.ndarray     # int32[m_a]
    assoc_a: np.ndarray     # int32[m_a]
    assoc_w: np.ndarray     # float32[m_a]

    @property
    def m_e(self) -> int:
        return int(self.edge_u.shape[0])

    @property
    def m_a(self) -> int:
        return int(self.assoc_u.shape[0])

    def u_degree_counts(self) -> np.ndarray:
        """|N(u)| for every u in U (number of incident edge entries)."""
        return np.bincount(self.edge_u, minlength=self.n_u)


# Workload shapes: the paper's Table 1 graphs are not available, so these
# seeded power-law graphs stand in for them.  Seeds are 1000 + index.
CONFIGS = {
    "tiny": BipartiteConfig("tiny", 2_000, 1_000, 20_000, 2.1, 2.1, 100, 5, 1.5, True, 1000),
    "m1": BipartiteConfig("m1", 1_000_000, 500_000, 20_000_000, 2.1, 2.1, 10_000, 20, 1.5, False, 1001),
    "serve5m": BipartiteConfig("serve5m", 5_000_000, 2_000_000, 100_000_000, 2.0, 2.0, 50_000, 30, 1.5,
                               False, 1003),
    "large20m": BipartiteConfig("large20m", 20_000_000, 10_000_000, 500_000_000, 2.1, 2.1, 50_000, 100, 1.3,
                                False, 1004),
    # Sizes of the paper's largest dataset (Amazon in Table 1: |U| 2.3M,
    # |V| 8.0M, |E| 22.5M, 800 attributes, 24.2M attribute entries); 10
    # attributes per U node give 23.0M entries.  Degree and popularity
    # exponents are not published; these reuse the other shapes' values.
    "amazon": BipartiteConfig("amazon", 2_300_000, 8_000_000, 22_500_000, 2.1, 2.1, 800, 10, 1.5, False, 1005),
}


def _draw_edges(cfg: BipartiteConfig) -> tuple[np.ndarray, np.ndarray]:
    rng_th = CounterRNG(cfg.seed, "theta")
    theta_u = _sample_cdf(_zipf_cdf(cfg.gamma_u, cfg.n_v), rng_th.uniform(cfg.n_u)).astype(np.int64) + 1
    theta_v = _sample_cdf(_zipf_cdf(cfg.gamma_v, cfg.n_u), rng_th.uniform(cfg.n_v)).astype(np.int64) + 1
    # Integer weights: node x appears theta[x] times in its urn, so a uniform
    # draw from the urn picks x with probability theta[x] / sum(theta).
    urn_u = np.repeat(np.arange(cfg.n_u, dtype=np.int64), theta_u)
    urn_v = np.repeat(np.arange(cfg.n_v, dtype=np.int64), theta_v)
    rng_e = CounterRNG(cfg.seed, "edges")
    keys = np.empty(0, dtype=np.int64)          # sorted distinct pairs u * n_v + v
    need = cfg.m_e
    rounds = 0
    while need > 0:
        k = int(need * 1.05) + 16
        u = urn_u[(rng_e.uniform(k) * urn_u.size).astype(np.int64)]
        v = urn_v[(rng_e.uniform(k) * urn_v.size).astype(np.int64)]
        cand = u * cfg.n_v + v
        uniq, first = np.unique(cand, return_index=True)
        if keys.size:
            pos = np.minimum(np.searchsorted(keys, uniq), keys.size - 1)
            fresh = keys[pos] != uniq
            uniq, first = uniq[fresh], first[fresh]
        if uniq.size > need:
            # Keep the earliest draws.
            keep = np.sort(np.argsort(first, kind="stable")[:need])
            uniq = uniq[keep]
        keys = np.sort(np.concatenate([keys, uniq]), kind="stable")
        need = cfg.m_e - keys.size
        rounds += 1
        if rounds > 500:
            raise RuntimeError("edge sampling did not reach the requested number of distinct pairs")
    # Every U node gets at least one edge.
    eu = keys // cfg.n_v
    deg = np.bincount(eu, minlength=cfg.n_u)
    lonely = np.nonzero(deg == 0)[0]
    if lonely.size:
        r = CounterRNG(cfg.seed, "lonely").uniform(lonely.size)
        fix_v = urn_v[(r * urn_v.size).astype(np.int64)]
        keys = np.sort(np.concatenate([keys, lonely * cfg.n_v + fix_v]), kind="stable")
    eu = keys // cfg.n_v
    ev = keys % cfg.n_v
    return eu.astype(np.int32), ev.astype(np.int32)


def _draw_attrs(cfg: BipartiteConfig) -> tuple[np.ndarray, np.ndarray]:
    c = min(cfg.attrs_per_node, cfg.n_attr)
    cdf = _zipf_cdf(cfg.attr_exponent, cfg.n_attr)
    rng = CounterRNG(cfg.seed, "attrs")
    # Rank r (0-based) maps to attribute id perm[r].
    perm = np.argsort(CounterRNG(cfg.seed, "attr_perm").bits(cfg.n_attr), kind="stable")
    n = cfg.n_u
    out = np.full((n, c), -1, dtype=np.int64)
    todo = np.arange(n, dtype=np.int64)
    width = 4 * c
    rounds = 0
    while todo.size:
        # Each pending node draws `width` ranks; its attributes are the first c
        # distinct ranks in draw order (sampling without replacement by rejection).
        m = todo.size
        draws = _sample_cdf(cdf, rng.uniform(m * width)).reshape(m, width).astype(np.int64)
        order = np.argsort(draws, axis=1, kind="stable")
        sd = np.take_along_axis(draws, order, axis=1)
        firstocc = np.ones_like(sd, dtype=bool)
        firstocc[:, 1:] = sd[:, 1:] != sd[:, :-1]
        # Draw positions of first occurrences; others pushed past the end.
        pos = np.where(firstocc, order, width)
        pos.sort(axis=1)
        ndist = firstocc.sum(axis=1)
        ok = ndist >= c
        sel = np.take_along_axis(draws, np.minimum(pos[:, :c], width - 1), axis=1)
        out[todo[ok]] = sel[ok]
        todo = todo[~ok]
        width *= 2
        rounds += 1
        if rounds > 30:
            raise RuntimeError("attribute sampling did not converge")
    au = np.repeat(np.arange(n, dtype=np.int64), c)
    aa = perm[out.reshape(-1)]
    order = np.lexsort((aa, au))
    return au[order].astype(np.int32), aa[order].astype(np.int32)


_NATIVE_LIB = None


def native_lib():
    """The multi-threaded generator (libsynth.so) if it is built, else None."""
    global _NATIVE_LIB
    if _NATIVE_LIB is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
        if not os.path.exists(path):
            return None
        lib = ctypes.CDLL(path)
        i64, u64, P = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.sn_draw_edges.restype = i64
        lib.sn_draw_edges.argtypes = [i64, i64, i64, P, P, u64, u64, u64, P, P]
        lib.sn_draw_attrs.restype = ctypes.c_int32
        lib.sn_draw_attrs.argtypes = [i64, i64, ctypes.c_int32, P, P, u64, P, P]
        lib.sn_uniform_f32.restype = None
        lib.sn_uniform_f32.argtypes = [u64, i64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P]
        _NATIVE_LIB = lib
    return _NATIVE_LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _draw_edges_native(lib, cfg: BipartiteConfig) -> tuple[np.ndarray, np.ndarray]:
    cdf_u = _zipf_cdf(cfg.gamma_u, cfg.n_v)
    cdf_v = _zipf_cdf(cfg.gamma_v, cfg.n_u)
    eu = np.empty(cfg.m_e + cfg.n_u, dtype=np.int32)
    ev = np.empty(cfg.m_e + cfg.n_u, dtype=np.int32)
    m = lib.sn_draw_edges(cfg.n_u, cfg.n_v, cfg.m_e, _p(cdf_u), _p(cdf_v), CounterRNG(cfg.seed, "theta").key,
                          CounterRNG(cfg.seed, "edges").key, CounterRNG(cfg.seed, "lonely").key, _p(eu), _p(ev))
    if m < 0:
        raise RuntimeError("edge sampling did not reach the requested number of distinct pairs")
    return eu[:m], ev[:m]


def _draw_attrs_native(lib, cfg: BipartiteConfig) -> tuple[np.ndarray, np.ndarray]:
    c = min(cfg.attrs_per_node, cfg.n_attr)
    cdf = _zipf_cdf(cfg.attr_exponent, cfg.n_attr)
    perm = np.ascontiguousarray(np.argsort(CounterRNG(cfg.seed, "attr_perm").bits(cfg.n_attr), kind="stable"),
                                dtype=np.int64)
    au = np.empty(cfg.n_u * c, dtype=np.int32)
    aa = np.empty(cfg.n_u * c, dtype=np.int32)
    if lib.sn_draw_attrs(cfg.n_u, cfg.n_attr, c, _p(cdf), _p(perm), CounterRNG(cfg.seed, "attrs").key,
                         _p(au), _p(aa)) < 0:
        raise RuntimeError("attribute sampling did not converge")
    return au, aa


def make_graph(cfg: BipartiteConfig | str, native: Optional[bool] = None) -> AttributedBipartiteGraph:
    """The graph of a configuration.  native: True forces libsynth.so, False
    the numpy definition, None uses libsynth.so when it is built."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    lib = native_lib() if native in (None, True) else None
    if native and lib is None:
        raise RuntimeError("libsynth.so is not built (paper_2512_11606_amd/build.py)")
    if lib is not None:
        eu, ev = _draw_edges_native(lib, cfg)
        au, aa = _draw_attrs_native(lib, cfg)
    else:
        eu, ev = _draw_edges(cfg)
        au, aa = _draw_attrs(cfg)
    if cfg.unit_weights:
        ew = np.ones(eu.shape[0], dtype=np.float32)
        aw = np.ones(au.shape[0], dtype=np.float32)
    elif lib is not None:
        ew = np.empty(eu.shape[0], dtype=np.float32)
        aw = np.empty(au.shape[0], dtype=np.float32)
        lib.sn_uniform_f32(CounterRNG(cfg.seed, "edge_w").key, ew.size, 0.5, 0.5, 0, _p(ew))
        lib.sn_uniform_f32(CounterRNG(cfg.seed, "assoc_w").key, aw.size, 1.0, -1.0, 1, _p(aw))
    else:
        ew = (0.5 + 0.5 * CounterRNG(cfg.seed, "edge_w").uniform(eu.shape[0])).astype(np.float32)
        aw = (1.0 - CounterRNG(cfg.seed, "assoc_w").uniform(au.shape[0])).astype(np.float32)
        # float32 rounding of 1 - u can give exactly 0 only if u rounds to 1: never, but clamp anyway.
        aw = np.maximum(aw, np.float32(np.finfo(np.float32).tiny))
    return AttributedBipartiteGraph(cfg, cfg.n_u, cfg.n_v, cfg.n_attr, eu, ev, ew, au, aa, aw)


def make_custom(n_u: int, n_v: int, m_e: int, n_attr: int, attrs_per_node: int, seed: int,
                gamma: float = 2.1, attr_exponent: float = 1.5, unit_weights: bool = False,
                native: Optional[bool] = None) -> AttributedBipartiteGraph:
    cfg = BipartiteConfig(f"custom{seed}", n_u, n_v, m_e, gamma, gamma, n_attr, attrs_per_node, attr_exponent,
                          unit_weights, seed)
    return make_graph(cfg, native=native)


def _compact(keep: np.ndarray) -> np.ndarray:
    """New ids of the kept entries of a mask (-1 for dropped ones)."""
    ids = np.cumsum(keep, dtype=np.int64) - 1
    return np.where(keep, ids, -1).astype(np.int64)


def _smallest_keys(keys: np.ndarray, k: int) -> np.ndarray:
    """Mask of the k entries with the smallest keys (64-bit random keys, so
    ties do not occur in practice)."""
    keep = np.zeros(keys.size, dtype=bool)
    if k >= keys.size:
        keep[:] = True
    elif k > 0:
        keep[np.argpartition(keys, k)[:k]] = True
    return keep


def sample_graph(g: AttributedBipartiteGraph, frac: float, mode: str, seed: int) -> AttributedBipartiteGraph:
    """A sampled subgraph in the manner of Exp-3's scalability graphs.

    mode "nodes": a seeded fraction of U (exactly round(frac |U|) nodes) with
    all their edges and attribute associations.  mode "edges": a seeded
    fraction of the edges (exactly round(frac |E|)), and the U nodes they
    touch with all their attribute associations.  In both, V nodes left
    without an edge are dropped and U / V ids are renumbered in their old
    order; the attribute ids and their count stay as they are."""
    if not (0.0 < frac <= 1.0):
        raise ValueError("frac must be in (0, 1]")
    if mode == "nodes":
        keep_u = _smallest_keys(CounterRNG(seed, "sample_u").bits(g.n_u), int(round(frac * g.n_u)))
        keep_e = keep_u[g.edge_u]
    elif mode == "edges":
        keep_e = _smallest_keys(CounterRNG(seed, "sample_e").bits(g.m_e), int(round(frac * g.m_e)))
        keep_u = np.zeros(g.n_u, dtype=bool)
        keep_u[g.edge_u[keep_e]] = True
    else:
        raise ValueError("mode must be 'nodes' or 'edges'")
    keep_v = np.zeros(g.n_v, dtype=bool)
    keep_v[g.edge_v[keep_e]] = True
    new_u, new_v = _compact(keep_u), _compact(keep_v)
    keep_a = keep_u[g.assoc_u]
    n_u, n_v = int(keep_u.sum()), int(keep_v.sum())
    cfg = dataclasses.replace(g.config, name=f"{g.config.name}-{mode}{frac:g}", n_u=n_u, n_v=n_v,
                              m_e=int(keep_e.sum()))
    return AttributedBipartiteGraph(cfg, n_u, n_v, g.n_attr,
                                    new_u[g.edge_u[keep_e]].astype(np.int32), new_v[g.edge_v[keep_e]].astype(np.int32),
                                    g.edge_w[keep_e], new_u[g.assoc_u[keep_a]].astype(np.int32),
                                    g.assoc_a[keep_a].copy(), g.assoc_w[keep_a])


def uniform_queries(g: AttributedBipartiteGraph, n: int, seed: int, distinct: bool = True) -> np.ndarray:
    """n source nodes drawn uniformly over U."""
    rng = CounterRNG(seed, "q_uniform")
    if distinct:
        if n > g.n_u:
            raise ValueError("more distinct queries than U nodes")
        order = np.argsort(rng.bits(g.n_u), kind="stable")
        return order[:n].astype(np.int32)
    return np.minimum((rng.uniform(n) * g.n_u).astype(np.int64), g.n_u - 1).astype(np.int32)


def degree_queries(g: AttributedBipartiteGraph, n: int, seed: int) -> np.ndarray:
    """n source nodes drawn with probability proportional to |N(u)| (with replacement)."""
    deg = g.u_degree_counts().astype(np.float64)
    c = np.cumsum(deg)
    c /= c[-1]
    return _sample_cdf(c, CounterRNG(seed, "q_degree").uniform(n)).astype(np.int32)


def mixed_batch_queries(g: AttributedBipartiteGraph, n: int, seed: int) -> np.ndarray:
    """n distinct sources: half uniform from the top 1% of U by |N(u)|, half uniform over U."""
    deg = g.u_degree_counts()
    order = np.argsort(-deg, kind="stable")
    top = order[: max(1, g.n_u // 100)]
    n_hub = min(n // 2, top.size)
    rng = CounterRNG(seed, "q_mixed")
    hubs = top[np.argsort(rng.bits(top.size), kind="stable")[:n_hub]]
    rest_pool = np.setdiff1d(np.arange(g.n_u), hubs)
    rest = rest_pool[np.argsort(rng.bits(rest_pool.size), kind="stable")[: n - n_hub]]
    out = np.concatenate([hubs, rest]).astype(np.int32)
    return out


def hub_queries(g: AttributedBipartiteGraph, n: int, seed: int) -> np.ndarray:
    """n sources drawn uniformly (with replacement) from the top 1% of U by |N(u)|."""
    deg = g.u_degree_counts()
    top = np.argsort(-deg, kind="stable")[: max(1, g.n_u // 100)]
    idx = np.minimum((CounterRNG(seed, "q_hub").uniform(n) * top.size).astype(np.int64), top.size - 1)
    return top[idx].astype(np.int32)


def summary(g: AttributedBipartiteGraph) -> dict:
    du = np.bincount(g.edge_u, minlength=g.n_u)
    dv = np.bincount(g.edge_v, minlength=g.n_v)
    da = np.bincount(g.assoc_a, minlength=g.n_attr)
    return {
        "n_u": g.n_u, "n_v": g.n_v, "n_attr": g.n_attr, "m_e": g.m_e, "m_a": g.m_a,
        "max_deg_u": int(du.max()), "max_deg_v": int(dv.max()), "max_deg_attr": int(da.max()),
        "isolated_u": int((du == 0).sum()), "isolated_v": int((dv == 0).sum()),
        "unused_attr": int((da == 0).sum()),
    }
