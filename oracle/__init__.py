"""CPU oracle for AHPP -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2512_11606_amd``): it reads the same seeded COO inputs and computes
everything itself, in double precision.

Pieces (each names the passage of arXiv 2512.11606 it follows):

* ``dense_PS`` / ``dense_PA`` / ``dense_P``: Eq. 1, Eq. 2 and the mixture of
  Def. 2, as dense matrices (tiny graphs).  ``dense_PS_literal`` and
  ``dense_PA_literal`` are the same equations as explicit sums over common
  neighbours / attributes, used to pin the matrix forms.
* ``exact_dense``: the matrix Pi = alpha (I - (1-alpha) P)^-1 whose row u is
  the AHPP vector of u (Def. 2 summed as a geometric series; the linear-system
  remark of Section 2.3).
* ``OracleGraph.power_series``: Def. 2 / Algorithm 1 (PI) as a truncated power
  series in C, with its certified tail (Section 3.2).
* ``OracleGraph.lambda_thm3``: Theorem 3, Eq. 6.
* ``OracleGraph.asrp`` / ``app`` / ``forward_push``: Algorithms 4, 3 and 2 in double
  precision; ``push_schedule``: the four schedules of Exp-2.
* ``topk``: the k most similar nodes (Exp-4/Exp-6 use of the scores).
* ``check_query``: Theorem 2's bound and sign, mass conservation, top-k band.

Parity unpinned: the exact intermediate values of ASRP, of Exp-2's other
schedules and of FP (iteration or push counts, n_p, the phase-switch round)
have no printed trace in the paper; only the final guarantees (Theorem 2,
and the per-node thresholds for APP / APP(S) / FP) and the invariant
(Lemma 2, after every round or push) are pinned.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ALPHA = 0.15   # restart probability default (Section 5.1 parameters)
BETA = 0.35    # attribute-jumping probability default (Section 5.1 parameters)


def pi_iterations(alpha: float, tol: float = 1e-12) -> int:
    """Smallest T with (1-alpha)^T <= tol: the PI round count of Section 3.2."""
    return int(math.ceil(math.log(tol) / math.log(1.0 - alpha)))


def lambda_iterations(n_u: int, alpha: float, slack: float = 0.01) -> int:
    """Smallest T with |U| (1-alpha)^T <= slack (the additive term of Eq. 6)."""
    return max(1, int(math.ceil(math.log(slack / n_u) / math.log(1.0 - alpha))))


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("switch_iteration", ctypes.c_int64), ("n_push", ctypes.c_int64),
                ("max_residual", ctypes.c_double), ("sum_residual", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.og_build.restype = P
    lib.og_build.argtypes = [i64, i64, i64, i64, P, P, P, i64, P, P, P]
    lib.og_free.argtypes = [P]
    lib.og_normalisers.argtypes = [P, P, P, P, P]
    lib.og_power_series.restype = ctypes.c_int
    lib.og_power_series.argtypes = [P, dbl, dbl, i32, ctypes.c_int, P, P, ctypes.c_int]
    lib.og_power_series_terms.restype = ctypes.c_int
    lib.og_power_series_terms.argtypes = [P, dbl, dbl, P, P, ctypes.c_int, ctypes.c_int]
    lib.og_l1.restype = dbl
    lib.og_l1.argtypes = [P, i64]
    lib.og_lambda_thm3.restype = dbl
    lib.og_lambda_thm3.argtypes = [P, dbl, dbl, ctypes.c_int, P, ctypes.c_int]
    lib.og_asrp.restype = ctypes.c_int
    lib.og_asrp.argtypes = [P, dbl, dbl, i32, dbl, dbl, i64, P, P, P]
    lib.og_asrp_hooked.restype = ctypes.c_int
    lib.og_asrp_hooked.argtypes = [P, dbl, dbl, i32, dbl, dbl, i64, P, P, P, P, P]
    lib.og_app.restype = ctypes.c_int
    lib.og_app.argtypes = [P, dbl, dbl, i32, dbl, i64, P, P, P]
    lib.og_forward_push.restype = ctypes.c_int
    lib.og_forward_push.argtypes = [P, dbl, dbl, i32, dbl, i64, P, P, P, P, P]
    lib.og_push_schedule.restype = ctypes.c_int
    lib.og_push_schedule.argtypes = [P, dbl, dbl, i32, dbl, dbl, i32, i64, P, P, P, P, P]
    lib.og_asrp_many.restype = ctypes.c_int
    lib.og_asrp_many.argtypes = [P, dbl, dbl, i32, P, dbl, dbl, i64, ctypes.c_int, P, P, P]
    lib.og_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


HOOK = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                        ctypes.c_void_p)


class _Hook:
    """A Python per-round hook as a C callback.  ctypes only prints an
    exception raised inside a callback, so the first one is kept (later
    rounds skip the hook) and raised again once the C call returns."""

    def __init__(self, hook, n: int):
        self.error = None
        self.ptr = None
        if hook is None:
            return

        def _cb(it, p, rr, user):
            if self.error is not None:
                return
            try:
                hook(int(it), np.ctypeslib.as_array(p, shape=(n,)).copy(),
                     np.ctypeslib.as_array(rr, shape=(n,)).copy())
            except BaseException as e:  # noqa: BLE001 - re-raised by reraise()
                self.error = e

        self._cb = HOOK(_cb)
        self.ptr = ctypes.cast(self._cb, ctypes.c_void_p)

    def reraise(self):
        if self.error is not None:
            raise self.error


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class PushStats:
    iterations: int
    switch_iteration: int
    n_push: int
    max_residual: float
    sum_residual: float


class OracleGraph:
    """Adjacency lists of one attributed bipartite graph, built by the C oracle."""

    def __init__(self, n_u, n_v, n_attr, edge_u, edge_v, edge_w, assoc_u, assoc_a, assoc_w):
        lib = _load()
        self.n_u, self.n_v, self.n_attr = int(n_u), int(n_v), int(n_attr)
        # A missing weight array means every weight is 1 (passed to C as NULL).
        self._keep = [None if x is None else np.ascontiguousarray(x, dtype=t) for x, t in
                      ((edge_u, np.int32), (edge_v, np.int32), (edge_w, np.float32),
                       (assoc_u, np.int32), (assoc_a, np.int32), (assoc_w, np.float32))]
        eu, ev, ew, au, aa, aw = self._keep
        self.m_e, self.m_a = int(eu.size), int(au.size)
        h = lib.og_build(self.n_u, self.n_v, self.n_attr, self.m_e, _ptr(eu), _ptr(ev), _ptr(ew),
                         self.m_a, _ptr(au), _ptr(aa), _ptr(aw))
        if not h:
            raise ValueError("oracle graph build failed (ids out of range?)")
        self._h = ctypes.c_void_p(h)
        self._keep = None

    @classmethod
    def from_graph(cls, g) -> "OracleGraph":
        return cls(g.n_u, g.n_v, g.n_attr, g.edge_u, g.edge_v, g.edge_w, g.assoc_u, g.assoc_a, g.assoc_w)

    def close(self):
        if getattr(self, "_h", None):
            _load().og_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def normalisers(self):
        d_u = np.zeros(self.n_u); d_v = np.zeros(self.n_v); s_u = np.zeros(self.n_u); t_a = np.zeros(self.n_attr)
        _load().og_normalisers(self._h, _ptr(d_u), _ptr(d_v), _ptr(s_u), _ptr(t_a))
        return d_u, d_v, s_u, t_a

    def power_series(self, source: int, alpha: float = ALPHA, beta: float = BETA, T: Optional[int] = None,
                     nthreads: int = 0, progress=None, every: int = 16):
        """Exact AHPP row of ``source`` (Def. 2) and the l1 bound of the dropped tail.

        With ``progress`` the T terms are summed ``every`` at a time (the same
        steps in the same order) and progress(terms_done, T) is called after
        each group."""
        T = pi_iterations(alpha) if T is None else T
        out = np.zeros(self.n_u)
        if progress is None:
            tail = ctypes.c_double(0.0)
            rc = _load().og_power_series(self._h, alpha, beta, int(source), int(T), _ptr(out), ctypes.byref(tail),
                                         int(nthreads))
            if rc != 0:
                raise ValueError("power_series: bad arguments")
            return out, tail.value
        if not 0 <= source < self.n_u or T < 0 or every < 1:
            raise ValueError("power_series: bad arguments")
        y = np.zeros(self.n_u)
        y[source] = 1.0
        done = 0
        while done < T:
            n = min(every, T - done)
            _load().og_power_series_terms(self._h, alpha, beta, _ptr(y), _ptr(out), int(n), int(nthreads))
            done += n
            progress(done, T)
        return out, _load().og_l1(_ptr(y), self.n_u)

    def lambda_thm3(self, alpha: float = ALPHA, beta: float = BETA, T: Optional[int] = None,
                    return_pi_T: bool = False, nthreads: int = 0):
        """Theorem 3 (Eq. 6): max_i pi_T(u_i) + |U| (1-alpha)^T."""
        T = lambda_iterations(self.n_u, alpha) if T is None else T
        pt = np.zeros(self.n_u) if return_pi_T else None
        lam = _load().og_lambda_thm3(self._h, alpha, beta, int(T), _ptr(pt), int(nthreads))
        return (lam, pt) if return_pi_T else lam

    def asrp(self, source: int, eps: float, lam: float, alpha: float = ALPHA, beta: float = BETA,
             max_iters: int = 1_000_000, hook=None):
        """Algorithm 4 in double precision: (reserve, U residues, stats)."""
        pi = np.zeros(self.n_u); r = np.zeros(self.n_u); st = _Stats()
        if hook is None:
            rc = _load().og_asrp(self._h, alpha, beta, int(source), eps, lam, int(max_iters), _ptr(pi), _ptr(r),
                                 ctypes.byref(st))
        else:
            hk = _Hook(hook, self.n_u)
            rc = _load().og_asrp_hooked(self._h, alpha, beta, int(source), eps, lam, int(max_iters), _ptr(pi),
                                        _ptr(r), ctypes.byref(st), hk.ptr, None)
            hk.reraise()
        if rc < 0:
            raise ValueError("asrp: bad arguments")
        stats = PushStats(st.iterations, st.switch_iteration, st.n_push, st.max_residual, st.sum_residual)
        return pi, r, stats, rc == 0

    def app(self, source: int, r_max: float, alpha: float = ALPHA, beta: float = BETA, max_iters: int = 1_000_000):
        """Algorithm 3 in double precision: (reserve, U residues, stats)."""
        pi = np.zeros(self.n_u); r = np.zeros(self.n_u); st = _Stats()
        rc = _load().og_app(self._h, alpha, beta, int(source), r_max, int(max_iters), _ptr(pi), _ptr(r),
                            ctypes.byref(st))
        if rc < 0:
            raise ValueError("app: bad arguments")
        return pi, r, PushStats(st.iterations, st.switch_iteration, st.n_push, st.max_residual,
                                st.sum_residual), rc == 0

    def forward_push(self, source: int, r_max: float, alpha: float = ALPHA, beta: float = BETA,
                     max_pushes: int = 100_000_000, hook=None):
        """Algorithm 2 (FP) in double precision, one node at a time from a FIFO
        queue: (reserve, U residues, stats, converged); stats.iterations counts
        node pushes.  hook(push, reserve, residues) runs after every push."""
        pi = np.zeros(self.n_u); r = np.zeros(self.n_u); st = _Stats()
        hk = _Hook(hook, self.n_u)
        rc = _load().og_forward_push(self._h, alpha, beta, int(source), r_max, int(max_pushes), _ptr(pi), _ptr(r),
                                     ctypes.byref(st), hk.ptr, None)
        hk.reraise()
        if rc < 0:
            raise ValueError("forward_push: bad arguments")
        stats = PushStats(st.iterations, st.switch_iteration, st.n_push, st.max_residual, st.sum_residual)
        return pi, r, stats, rc == 0

    def push_schedule(self, source: int, eps: float, lam: float, schedule: int, alpha: float = ALPHA,
                      beta: float = BETA, max_iters: int = 1_000_000, hook=None):
        """Exp-2's schedules (0 ASRP, 1 APP, 2 APP(S), 3 APP(E)) in double
        precision: (reserve, U residues, stats, converged)."""
        pi = np.zeros(self.n_u); r = np.zeros(self.n_u); st = _Stats()
        hk = _Hook(hook, self.n_u)
        rc = _load().og_push_schedule(self._h, alpha, beta, int(source), eps, lam, int(schedule), int(max_iters),
                                      _ptr(pi), _ptr(r), ctypes.byref(st), hk.ptr, None)
        hk.reraise()
        if rc < 0:
            raise ValueError("push_schedule: bad arguments")
        stats = PushStats(st.iterations, st.switch_iteration, st.n_push, st.max_residual, st.sum_residual)
        return pi, r, stats, rc == 0

    def asrp_many(self, sources: Sequence[int], eps: float, lam: float, alpha: float = ALPHA, beta: float = BETA,
                  nthreads: int = 0, keep_pi: bool = False, max_iters: int = 1_000_000):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        pi = np.zeros((src.size, self.n_u)) if keep_pi else None
        st = (_Stats * max(1, src.size))()
        secs = np.zeros(max(1, src.size))
        bad = _load().og_asrp_many(self._h, alpha, beta, int(src.size), _ptr(src), eps, lam, int(max_iters),
                                   int(nthreads), _ptr(pi), ctypes.cast(st, ctypes.c_void_p), _ptr(secs))
        stats = [PushStats(s.iterations, s.switch_iteration, s.n_push, s.max_residual, s.sum_residual)
                 for s in st[: src.size]]
        self.last_secs = secs[: src.size]
        return pi, stats, bad


def max_threads() -> int:
    return int(_load().og_max_threads())


# ---------------------------------------------------------------------------
# Dense forms for tiny graphs (numpy, float64).
# ---------------------------------------------------------------------------

def _dense_w(n_rows, n_cols, rows, cols, w):
    M = np.zeros((n_rows, n_cols))
    rows = np.asarray(rows)
    vals = np.ones(rows.shape) if w is None else np.asarray(w, dtype=np.float64)
    np.add.at(M, (rows, np.asarray(cols)), vals)
    return M


def dense_PS(g) -> np.ndarray:
    """Eq. 1: P_S[i,j] = sum_{v in N(i) and N(j)} w(i,v)/d(i) * w(v,j)/d(v), as D_U^-1 W D_V^-1 W^T."""
    W = _dense_w(g.n_u, g.n_v, g.edge_u, g.edge_v, g.edge_w)
    d_u = W.sum(axis=1)
    d_v = W.sum(axis=0)
    inv_u = np.divide(1.0, d_u, out=np.zeros_like(d_u), where=d_u > 0)
    inv_v = np.divide(1.0, d_v, out=np.zeros_like(d_v), where=d_v > 0)
    return (inv_u[:, None] * W) @ (inv_v[:, None] * W.T)


def dense_PA(g) -> np.ndarray:
    """Eq. 2: P_A[i,j] = sum_{a in A(i) and A(j)} w(i,a)/s(i) * w(j,a)/t(a)."""
    X = _dense_w(g.n_u, g.n_attr, g.assoc_u, g.assoc_a, g.assoc_w)
    s_u = X.sum(axis=1)
    t_a = X.sum(axis=0)
    inv_s = np.divide(1.0, s_u, out=np.zeros_like(s_u), where=s_u > 0)
    inv_t = np.divide(1.0, t_a, out=np.zeros_like(t_a), where=t_a > 0)
    return (inv_s[:, None] * X) @ (inv_t[:, None] * X.T)


def dense_PS_literal(g) -> np.ndarray:
    """Eq. 1 as written: a sum over common neighbours v, one pair at a time (small graphs only)."""
    nbr = [dict() for _ in range(g.n_u)]
    ew = np.ones(len(g.edge_u)) if g.edge_w is None else g.edge_w
    for u, v, w in zip(g.edge_u.tolist(), g.edge_v.tolist(), ew.tolist()):
        nbr[u][v] = nbr[u].get(v, 0.0) + float(w)
    d_u = [sum(x.values()) for x in nbr]
    d_v = [0.0] * g.n_v
    for x in nbr:
        for v, w in x.items():
            d_v[v] += w
    P = np.zeros((g.n_u, g.n_u))
    for i in range(g.n_u):
        for j in range(g.n_u):
            for v in set(nbr[i]) & set(nbr[j]):
                P[i, j] += nbr[i][v] / d_u[i] * nbr[j][v] / d_v[v]
    return P


def dense_PA_literal(g) -> np.ndarray:
    """Eq. 2 as written: a sum over common attributes a (small graphs only)."""
    att = [dict() for _ in range(g.n_u)]
    aw = np.ones(len(g.assoc_u)) if g.assoc_w is None else g.assoc_w
    for u, a, w in zip(g.assoc_u.tolist(), g.assoc_a.tolist(), aw.tolist()):
        att[u][a] = att[u].get(a, 0.0) + float(w)
    s_u = [sum(x.values()) for x in att]
    t_a = [0.0] * g.n_attr
    for x in att:
        for a, w in x.items():
            t_a[a] += w
    P = np.zeros((g.n_u, g.n_u))
    for i in range(g.n_u):
        for j in range(g.n_u):
            for a in set(att[i]) & set(att[j]):
                P[i, j] += att[i][a] / s_u[i] * att[j][a] / t_a[a]
    return P


def dense_P(g, beta: float = BETA) -> np.ndarray:
    """Def. 2: P = (1 - beta) P_S + beta P_A."""
    return (1.0 - beta) * dense_PS(g) + beta * dense_PA(g)


def exact_dense(g, alpha: float = ALPHA, beta: float = BETA) -> np.ndarray:
    """Pi with Pi[i, j] = pi(u_i, u_j) = alpha * ((I - (1-alpha) P)^-1)[i, j] (Def. 2)."""
    P = dense_P(g, beta)
    n = P.shape[0]
    return alpha * np.linalg.solve(np.eye(n) - (1.0 - alpha) * P, np.eye(n))


def topk(pi: np.ndarray, k: int, exclude: int = -1):
    """k largest scores with pi > 0, ties by smaller id, ``exclude`` left out."""
    ids = np.arange(pi.size)
    keep = pi > 0
    if 0 <= exclude < pi.size:
        keep[exclude] = False
    ids = ids[keep]
    vals = pi[keep]
    order = np.lexsort((ids, -vals))[:k]
    return ids[order], vals[order]


@dataclass
class QueryCheck:
    max_abs_err: float
    max_over: float          # max(pi_hat - pi), must stay <= tol
    min_value: float
    mass_err: Optional[float]
    topk_ok: Optional[bool]
    ok: bool
    detail: str


def check_query(pi_exact: np.ndarray, pi_hat: np.ndarray, eps: float, tol: float = 1e-6,
                resid: Optional[np.ndarray] = None, mass_tol: float = 1e-5, k: int = 0, source: int = -1,
                topk_ids: Optional[np.ndarray] = None) -> QueryCheck:
    """Acceptance of one approximate query against the exact vector.

    * Theorem 2 bound: |pi - pi_hat| <= eps + tol everywhere.
    * Theorem 2 sign:  pi_hat >= 0 and pi_hat <= pi + tol.
    * Lemma 2 summed over i (rows of Pi sum to one without dangling nodes):
      |sum pi_hat + sum r - 1| <= mass_tol when residues are given.
    * Top-k: with pi_(k) the exact k-th score and d = eps + tol, every node
      scoring above pi_(k) + 2d must be returned, none below pi_(k) - 2d.
    """
    pi_exact = np.asarray(pi_exact, dtype=np.float64)
    pi_hat = np.asarray(pi_hat, dtype=np.float64)
    err = np.abs(pi_exact - pi_hat)
    max_err = float(err.max()) if err.size else 0.0
    over = float((pi_hat - pi_exact).max()) if err.size else 0.0
    mn = float(pi_hat.min()) if err.size else 0.0
    msgs = []
    ok = True
    if not max_err <= eps + tol:
        ok = False
        msgs.append(f"max |err| {max_err:.3e} > eps+tol {eps + tol:.3e} at {int(err.argmax())}")
    if not over <= tol:
        ok = False
        msgs.append(f"pi_hat exceeds pi by {over:.3e}")
    if not mn >= 0:
        ok = False
        msgs.append(f"negative pi_hat {mn:.3e}")
    mass_err = None
    if resid is not None:
        mass_err = abs(float(pi_hat.sum()) + float(np.asarray(resid, dtype=np.float64).sum()) - 1.0)
        if not mass_err <= mass_tol:
            ok = False
            msgs.append(f"mass error {mass_err:.3e}")
    tk_ok = None
    if k > 0 and topk_ids is not None:
        tk_ok = topk_band_ok(pi_exact, np.asarray(topk_ids), k, eps + tol, source)
        if not tk_ok:
            ok = False
            msgs.append("top-k outside the band")
    return QueryCheck(max_err, over, mn, mass_err, tk_ok, ok, "; ".join(msgs))


def topk_band_ok(pi_exact: np.ndarray, got_ids: np.ndarray, k: int, delta: float, source: int = -1) -> bool:
    """Top-k acceptance band (the top-k use of the scores in Exp-6, Section 5.3).

    With pi_(k) the exact k-th score (source left out) and delta the allowed
    error of every score (Theorem 2's eps plus the float tolerance):
    * at most k distinct ids, the source not among them;
    * every node scoring above pi_(k) + 2 delta is listed, none below
      pi_(k) - 2 delta (swaps inside the band are allowed);
    * a list shorter than k names every node scoring above delta: such a
      node's approximate score is above zero, so it was a candidate.
    """
    ex = np.asarray(pi_exact, dtype=np.float64).copy()
    if 0 <= source < ex.size:
        ex[source] = -np.inf
    ids = [int(i) for i in np.asarray(got_ids).tolist()]
    got = set(ids)
    if len(got) != len(ids) or len(ids) > k:
        return False
    if source in got or any(i < 0 or i >= ex.size for i in got):
        return False
    order = np.lexsort((np.arange(ex.size), -ex))
    kth = ex[order[min(k, ex.size) - 1]]
    must = np.nonzero(ex > kth + 2 * delta)[0]
    banned = np.nonzero((ex < kth - 2 * delta) & np.isfinite(ex))[0]
    if any(int(i) not in got for i in must):
        return False
    if any(int(i) in got for i in banned):
        return False
    if len(ids) < k and any(int(i) not in got for i in np.nonzero(ex > delta)[0]):
        return False
    return True
