"""The batched engine's transport rounding, modelled densely in FP64 on small
graphs (CPU only; no GPU code is used).

The batched kernels keep residues and reserves in float32 but hand on, from
one half-step to the other, only each value rounded toward zero to 8
significant bits (bfloat16), keeping the exact remainder: a U node above the
threshold pushes t8(r) and keeps r - t8(r); a V / attribute row hands on
t8(z) and carries z - t8(z) into its next round.  This model follows those
steps with the dense matrices of Eq. 1 / Eq. 2 and checks what makes the
scheme correct:

* Lemma 2 (Eq. 5) holds after every round once the carries count as the
  residues a push of them would leave: pi(s, .) = pi_hat + r' Pi with
  r'(u) = r(u) + sum_x w(u,x) c(x);
* the carried part never exceeds 2^-7 of what was pulled in, so
  r' <= r + 2^-7 s, the bound the stop rule tests against eps / lambda;
* at the stop, Theorem 2's bound 0 <= pi - pi_hat <= eps holds.
"""

import numpy as np
import pytest

import oracle as O
from paper_2512_11606_amd import synth


def t8(v):
    """v rounded toward zero to 8 significant bits (what keeping the top 16
    bits of a float32 does to its value)."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)
    return np.ldexp(np.floor(m * 256.0) / 256.0, e)


def test_t8_pins():
    assert t8(1.0) == 1.0
    assert t8(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    assert t8(1.0 + 2.0 ** -8) == 1.0
    assert t8(0.0) == 0.0
    x = np.random.default_rng(3).uniform(1e-30, 10.0, 10000)
    q = t8(x)
    assert np.all(q <= x) and np.all(x - q < 2.0 ** -7 * q)
    # the same as keeping the top 16 bits of the float32 pattern
    f = x.astype(np.float32)
    bits = (f.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    assert np.array_equal(bits, t8(f.astype(np.float64)))


def _mats(g, alpha, beta):
    """Back weights B[x, u] = w'(u, x) (the U push split by Eq. 1 / Eq. 2 with
    (1 - alpha) folded in), row scales 1/d(v), 1/t(a), and raw forward
    weights F[u, x] = w(u, x); x runs over V, then the attributes."""
    W = O._dense_w(g.n_u, g.n_v, g.edge_u, g.edge_v, g.edge_w)
    X = O._dense_w(g.n_u, g.n_attr, g.assoc_u, g.assoc_a, g.assoc_w)
    d_u, d_v, s_u, t_a = W.sum(1), W.sum(0), X.sum(1), X.sum(0)
    inv = lambda a: np.divide(1.0, a, out=np.zeros_like(a), where=a > 0)  # noqa: E731
    B = np.vstack([((1 - beta) * (1 - alpha) * W * inv(d_u)[:, None]).T,
                   (beta * (1 - alpha) * X * inv(s_u)[:, None]).T])
    inv_b = np.concatenate([inv(d_v), inv(t_a)])
    F = np.hstack([W, X])
    deg = (W > 0).sum(1) + (X > 0).sum(1)
    row_len = np.concatenate([(W > 0).sum(0), (X > 0).sum(0)])
    return B, inv_b, F, deg, row_len


def run_model(g, src, eps, lam, alpha=O.ALPHA, beta=O.BETA, Pi=None, max_rounds=10000):
    B, inv_b, F, deg, row_len = _mats(g, alpha, beta)
    n_u = g.n_u
    eps_f = eps / lam
    r = np.zeros(n_u); r[src] = 1.0
    pi = np.zeros(n_u)
    c = np.zeros(B.shape[0])
    theta, theta_q, phase, n_p = eps_f, 0.0, 1, 0
    budget = 2.0 * (g.m_e + g.m_a)
    worst_inv = 0.0
    for it in range(1, max_rounds + 1):
        q = np.where(r > theta_q, t8(r), 0.0)          # what U pushes this round (Q)
        z = c + inv_b * (B @ q)                          # V / attribute residues over d(v), t(a)
        zh = t8(z)
        c = z - zh                                       # carried to the next round
        s = F @ zh                                       # pulled into U
        assert np.all(c <= 2.0 ** -7 * zh + 1e-300)
        pi += alpha * q
        r = r - q + s
        n_p += int(deg[q > 0].sum() + row_len[z > 0].sum())
        if Pi is not None:
            r_full = r + F @ c                           # residues once every carry is pushed
            assert np.all(r_full <= r + 2.0 ** -7 * s + 1e-18)
            worst_inv = max(worst_inv, float(np.abs(pi + r_full @ Pi - Pi[src]).max()))
        m = float((r + 2.0 ** -7 * s).max())
        theta_q = theta
        if not m > eps_f:
            return pi, r, c, F, it, worst_inv
        if phase == 1 and n_p >= budget * max(0.0, np.log(m / eps_f) / np.log(1.0 / (1.0 - alpha))):
            phase, theta = 2, 0.0
    raise AssertionError("model did not stop")


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_transport_keeps_lemma2_and_theorem2(tiny_graph, tiny_oracle, tiny_Pi, eps):
    lam = tiny_oracle.lambda_thm3()
    for src in (0, 17, 1999):
        pi, r, c, F, rounds, worst = run_model(tiny_graph, src, eps, lam, Pi=tiny_Pi)
        assert worst < 1e-12, worst
        err = tiny_Pi[src] - pi
        assert err.min() >= -1e-13 and err.max() <= eps, (src, err.min(), err.max())
        assert abs(pi.sum() + (r + F @ c).sum() - 1.0) < 1e-12


def test_transport_on_a_weighted_graph():
    g = synth.make_custom(300, 120, 2000, 20, 4, seed=77, unit_weights=False)
    og = O.OracleGraph.from_graph(g)
    Pi = O.exact_dense(g)
    lam = og.lambda_thm3()
    for src in (3, 150):
        pi, r, c, F, rounds, worst = run_model(g, src, 1e-7, lam, Pi=Pi)
        assert worst < 1e-12
        err = Pi[src] - pi
        assert err.min() >= -1e-13 and err.max() <= 1e-7
        # the full-push rounds of Algorithm 4 need about as many rounds
        _, _, st, ok = og.asrp(src, 1e-7, lam)
        assert ok and abs(rounds - st.iterations) <= 3, (rounds, st.iterations)


def test_dropping_the_carries_breaks_lemma2(tiny_graph, tiny_Pi):
    """A plausible slip, forgetting the carried remainders, loses mass and
    breaks the invariant; the pins above would catch it."""
    B, inv_b, F, deg, row_len = _mats(tiny_graph, O.ALPHA, O.BETA)
    r = np.zeros(tiny_graph.n_u); r[5] = 1.0
    pi = np.zeros_like(r)
    for _ in range(3):
        q = t8(r)
        zh = t8(inv_b * (B @ q))
        pi += O.ALPHA * q
        r = r - q + F @ zh
    assert np.abs(pi + r @ tiny_Pi - tiny_Pi[5]).max() > 1e-6
