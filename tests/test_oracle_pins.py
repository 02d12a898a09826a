"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses a value the
paper prints, a closed form derived by hand, an independent characterisation
(Perron vector, random walks), an invariant stated by a lemma or theorem, or
brute force.  The planted-mistake tests at the end show that plausible slips
in the formulas fail at least one pin.
"""

import json
import math
import os
import types

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from paper_2512_11606_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make(n_u, n_v, n_attr, edges, assoc, ew=None, aw=None):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    a = np.asarray(assoc, dtype=np.int64).reshape(-1, 2)
    return types.SimpleNamespace(
        n_u=n_u, n_v=n_v, n_attr=n_attr,
        edge_u=e[:, 0].astype(np.int32), edge_v=e[:, 1].astype(np.int32),
        edge_w=np.ones(len(e), np.float32) if ew is None else np.asarray(ew, np.float32),
        assoc_u=a[:, 0].astype(np.int32), assoc_a=a[:, 1].astype(np.int32),
        assoc_w=np.ones(len(a), np.float32) if aw is None else np.asarray(aw, np.float32))


def complete_bipartite(m, n, private_attr):
    edges = [(i, j) for i in range(m) for j in range(n)]
    if private_attr:
        return make(m, n, m, edges, [(i, i) for i in range(m)])
    return make(m, n, 1, edges, [(i, 0) for i in range(m)])


def small_weighted(seed=5, n_u=40, n_v=25, m_e=160, n_attr=9, c=3):
    return synth.make_custom(n_u, n_v, m_e, n_attr, c, seed=seed, unit_weights=False)


# ---------------------------------------------------------------- Eq. 1 / Eq. 2

def test_example1_structure_transition():
    """Section 2.1, Example 1: P_S[u1,u2] = 3/8 and P_S[u1,u3] = 1/8."""
    fx = json.load(open(os.path.join(GOLDEN, "example1.json")))
    g = make(fx["n_u"], fx["n_v"], fx["n_attr"], fx["edges"], fx["assoc"])
    for PS in (O.dense_PS(g), O.dense_PS_literal(g)):
        assert PS[0, 1] == pytest.approx(fx["expected"]["PS_u1_u2"], abs=1e-15)
        assert PS[0, 2] == pytest.approx(fx["expected"]["PS_u1_u3"], abs=1e-15)
        # The rest of u1's row follows from the stated adjacency: v2 also
        # reaches u4 (1/8) and u1 itself gets 1/2*1/2 + 1/2*1/4 = 3/8.
        assert PS[0].tolist() == pytest.approx([0.375, 0.375, 0.125, 0.125], abs=1e-15)


def test_literal_sums_equal_matrix_forms():
    g = small_weighted()
    assert np.allclose(O.dense_PS(g), O.dense_PS_literal(g), atol=1e-14, rtol=0)
    assert np.allclose(O.dense_PA(g), O.dense_PA_literal(g), atol=1e-14, rtol=0)


def test_transition_rows_are_stochastic(tiny_graph):
    """Without dangling nodes every row of P_S, P_A (Eq. 1, Eq. 2) sums to one."""
    for P in (O.dense_PS(tiny_graph), O.dense_PA(tiny_graph)):
        assert np.abs(P.sum(axis=1) - 1).max() < 1e-12
        assert P.min() >= 0


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("m,n", [(4, 3), (2, 5), (7, 2)])
def test_closed_form_single_shared_attribute(m, n):
    """K_{m,n}, unit weights, one attribute shared by all: P = J/m, so
    pi(u,u) = alpha + (1-alpha)/m and pi(u,j) = (1-alpha)/m."""
    a = O.ALPHA
    g = complete_bipartite(m, n, private_attr=False)
    og = O.OracleGraph.from_graph(g)
    pi, _ = og.power_series(0)
    want = np.full(m, (1 - a) / m)
    want[0] = a + (1 - a) / m
    assert np.abs(pi - want).max() < 1e-12
    assert np.abs(O.exact_dense(g)[0] - want).max() < 1e-13
    if m == 4:
        assert pi[0] == pytest.approx(0.3625, abs=1e-12)
        assert pi[1] == pytest.approx(0.2125, abs=1e-12)


@pytest.mark.parametrize("m", [2, 3, 6])
@pytest.mark.parametrize("beta", [0.35, 0.8])
def test_closed_form_private_attributes(m, beta):
    """K_{m,n} with a private attribute per U node: P = (1-b) J/m + b I, so
    pi(u,u) = 1/m + a(1-1/m)/(1-(1-a)b) and pi(u,j) = 1/m - a/(m(1-(1-a)b))."""
    a = O.ALPHA
    g = complete_bipartite(m, 3, private_attr=True)
    og = O.OracleGraph.from_graph(g)
    pi, _ = og.power_series(0, beta=beta)
    den = 1 - (1 - a) * beta
    want = np.full(m, 1 / m - a / (m * den))
    want[0] = 1 / m + a * (1 - 1 / m) / den
    assert np.abs(pi - want).max() < 1e-12
    if m == 2 and beta == 0.35:
        assert pi[0] == pytest.approx(0.6067616, abs=5e-8)
        assert pi[1] == pytest.approx(0.3932384, abs=5e-8)


# ---------------------------------------------------------------- exact AHPP

def test_power_series_matches_dense_solve(tiny_oracle, tiny_Pi):
    for s in (0, 1, 777, 1999):
        pi, tail = tiny_oracle.power_series(s)
        assert np.abs(pi - tiny_Pi[s]).max() < 1e-12
        assert tail < 1e-12


def test_power_series_in_groups_equals_one_call(tiny_oracle, tiny_Pi):
    """Summed a few terms at a time (with progress reports) the series takes
    the same steps: the same row and tail bit for bit, still the dense solve."""
    seen = []
    for every in (1, 7, 64, 1000):
        seen.clear()
        pi, tail = tiny_oracle.power_series(777, progress=lambda d, t: seen.append((d, t)), every=every)
        ref, ref_tail = tiny_oracle.power_series(777)
        assert np.array_equal(pi, ref) and tail == ref_tail
        assert np.abs(pi - tiny_Pi[777]).max() < 1e-12
        assert seen[-1][0] == seen[-1][1] and all(a[0] < b[0] for a, b in zip(seen, seen[1:]))
    with pytest.raises(ValueError):
        tiny_oracle.power_series(-1, progress=print)


def test_power_series_weighted_matches_dense_solve():
    g = small_weighted()
    og = O.OracleGraph.from_graph(g)
    for beta in (0.0, 0.35, 1.0):
        Pi = O.exact_dense(g, beta=beta)
        for s in range(0, g.n_u, 7):
            pi, _ = og.power_series(s, beta=beta)
            assert np.abs(pi - Pi[s]).max() < 1e-12


def test_pi_is_perron_vector_of_restart_chain():
    """Independent characterisation: pi_u is the stationary distribution of the
    chain that follows P with probability 1-alpha and jumps to u with
    probability alpha (the PageRank / Google-matrix view of Section 3.2)."""
    g = small_weighted(seed=9)
    og = O.OracleGraph.from_graph(g)
    P = O.dense_P(g)
    for s in (0, 5, 17):
        G = (1 - O.ALPHA) * P
        G[:, s] += O.ALPHA
        w, vl = scipy.linalg.eig(G, left=True, right=False)
        k = int(np.argmin(np.abs(w - 1)))
        stat = np.real(vl[:, k])
        stat = stat / stat.sum()
        pi, _ = og.power_series(s)
        assert np.abs(pi - stat).max() < 1e-10


def test_truncation_tail_is_exact_without_dangling(tiny_oracle):
    """Rows of P are stochastic, so ||(1-alpha)^T e_u P^T||_1 = (1-alpha)^T."""
    for T in (5, 40):
        _, tail = tiny_oracle.power_series(3, T=T)
        assert tail == pytest.approx((1 - O.ALPHA) ** T, rel=1e-12)
    assert O.pi_iterations(0.15) == 171


def test_reversibility_at_pure_structure_and_pure_attributes():
    """beta=0 is HPP (PPR on P_S), reversible w.r.t. d; beta=1 is reversible
    w.r.t. s.  A genuine mixture is not reversible w.r.t. either."""
    g = small_weighted(seed=3)
    og = O.OracleGraph.from_graph(g)
    d_u, _, s_u, _ = og.normalisers()
    for beta, wt in ((0.0, d_u), (1.0, s_u)):
        Pi = O.exact_dense(g, beta=beta)
        M = wt[:, None] * Pi
        assert np.abs(M - M.T).max() < 1e-13
    Pi = O.exact_dense(g, beta=0.35)
    for wt in (d_u, s_u):
        M = wt[:, None] * Pi
        assert np.abs(M - M.T).max() > 1e-6


def test_random_walk_interpretation():
    """Lemma 1: pi(u, .) is the stopping distribution of the walk that stops
    with probability alpha, otherwise takes a structure step (prob. 1-beta:
    u -> v ~ w(u,v), v -> u' ~ w(v,u')) or an attribute step (prob. beta:
    u -> a ~ w(u,a), a -> u' ~ w(u',a)).  Walks are simulated from the COO
    lists alone; Hoeffding bound with failure probability 1e-6 per entry."""
    g = small_weighted(seed=11, n_u=20, n_v=12, m_e=70, n_attr=5, c=2)
    og = O.OracleGraph.from_graph(g)
    rng = np.random.default_rng(1234)
    src, n_walks = 4, 200_000

    def step_table(rows, cols, w, n_rows):
        out = []
        for r in range(n_rows):
            m = rows == r
            p = w[m].astype(np.float64)
            out.append((cols[m], np.cumsum(p) / p.sum()))
        return out

    u2v = step_table(g.edge_u, g.edge_v, g.edge_w, g.n_u)
    v2u = step_table(g.edge_v, g.edge_u, g.edge_w, g.n_v)
    u2a = step_table(g.assoc_u, g.assoc_a, g.assoc_w, g.n_u)
    a2u = step_table(g.assoc_a, g.assoc_u, g.assoc_w, g.n_attr)

    def pick(tab, cur):
        out = np.empty_like(cur)
        r = rng.random(cur.size)
        for x in np.unique(cur):
            m = cur == x
            c, cdf = tab[x]
            out[m] = c[np.minimum(np.searchsorted(cdf, r[m], side="right"), len(c) - 1)]
        return out

    pos = np.full(n_walks, src)
    alive = np.ones(n_walks, bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        stop = rng.random(idx.size) < O.ALPHA
        alive[idx[stop]] = False
        idx = idx[~stop]
        if not idx.size:
            break
        attr = rng.random(idx.size) < O.BETA
        si, ai = idx[~attr], idx[attr]
        if si.size:
            pos[si] = pick(v2u, pick(u2v, pos[si]))
        if ai.size:
            pos[ai] = pick(a2u, pick(u2a, pos[ai]))
    emp = np.bincount(pos, minlength=g.n_u) / n_walks
    pi, _ = og.power_series(src)
    band = math.sqrt(math.log(2 * g.n_u / 1e-6) / (2 * n_walks))
    assert np.abs(emp - pi).max() < band


# ---------------------------------------------------------------- push algorithms

def _small_dense_case():
    g = small_weighted(seed=21, n_u=60, n_v=30, m_e=240, n_attr=8, c=3)
    return g, O.OracleGraph.from_graph(g), O.exact_dense(g)


def test_lemma2_invariant_after_every_round():
    """Lemma 2 (Eq. 5): pi(u,i) = pi_hat(u,i) + sum_j r(u,j) pi(u_j,i) after
    every round of Algorithm 4, and mass pi_hat + r sums to one."""
    g, og, Pi = _small_dense_case()
    lam = og.lambda_thm3()
    seen = []

    def hook(it, pi_hat, r):
        lhs = Pi[7]
        rhs = pi_hat + r @ Pi
        seen.append(it)
        assert np.abs(lhs - rhs).max() < 1e-13
        assert abs(pi_hat.sum() + r.sum() - 1) < 1e-13

    _, _, st, ok = og.asrp(7, 1e-6, lam, hook=hook)
    assert ok and seen == list(range(1, st.iterations + 1)) and st.iterations > 3


@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-6])
def test_asrp_guarantee_theorem2(tiny_oracle, tiny_Pi, eps):
    """Theorem 2 with lambda from Theorem 3: 0 <= pi - pi_hat <= eps."""
    lam = tiny_oracle.lambda_thm3()
    for s in (0, 123, 1500):
        pi_hat, r, st, ok = tiny_oracle.asrp(s, eps, lam)
        assert ok
        diff = tiny_Pi[s] - pi_hat
        assert diff.min() >= -1e-14
        assert diff.max() <= eps
        assert st.max_residual <= eps / lam
        assert abs(pi_hat.sum() + r.sum() - 1) < 1e-12


def test_asrp_synchronous_phase_is_reached():
    """The budget test of Algorithm 4 does switch to synchronous push (threshold 0)."""
    g, og, Pi = _small_dense_case()
    lam = og.lambda_thm3()
    _, _, st, ok = og.asrp(3, 1e-9, lam)
    assert ok and st.switch_iteration > 0


def test_paper_experiment_lambda_can_break_the_bound(tiny_oracle, tiny_Pi):
    """Reading of Theorem 2: the proof needs lambda >= the largest column sum
    of Pi.  The per-query choice lambda = max_i pi(u, u_i) used in Exp-1 can
    violate the eps bound on a hub-heavy graph; Theorem 3's lambda does not."""
    eps = 1e-6
    pi_hat, _, _, _ = tiny_oracle.asrp(0, eps, float(tiny_Pi[0].max()))
    assert np.abs(tiny_Pi[0] - pi_hat).max() > eps


def test_app_guarantee():
    """Algorithm 3 with r_max = eps/(|E| + |E_A|) meets the eps bound."""
    g, og, Pi = _small_dense_case()
    eps = 1e-5
    pi_hat, r, st, ok = og.app(11, eps / (og.m_e + og.m_a))
    assert ok
    assert 0 <= (Pi[11] - pi_hat).min() + 1e-15
    assert (Pi[11] - pi_hat).max() <= eps


SCHEDULES = (0, 1, 2, 3)  # ASRP, APP, APP(S), APP(E)


def test_schedules_reduce_to_the_two_algorithms():
    """Exp-2's schedule 0 is Algorithm 4 and schedule 1 is Algorithm 3 with
    r_max = eps/(|E| + |E_A|): identical reserves, residues and counts."""
    g, og, Pi = _small_dense_case()
    lam = og.lambda_thm3()
    eps = 1e-6
    a = og.asrp(5, eps, lam)
    b = og.push_schedule(5, eps, lam, 0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    c = og.app(5, eps / (og.m_e + og.m_a))
    d = og.push_schedule(5, eps, lam, 1)
    assert np.array_equal(c[0], d[0]) and np.array_equal(c[1], d[1])
    assert c[2].iterations == d[2].iterations and c[2].n_push == d[2].n_push


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_schedule_invariant_and_bound(schedule):
    """Every schedule keeps Lemma 2 after every round (it only reorders which
    residues are pushed) and ends within eps of the exact row: APP(E) by
    Theorem 2 (its stop rule is max r <= eps/lambda), APP and APP(S) by
    Algorithm 3's residue threshold (they stop under it)."""
    g, og, Pi = _small_dense_case()
    lam = og.lambda_thm3()
    eps = 1e-5
    rounds = []

    def hook(it, pi_hat, r):
        rounds.append(it)
        assert np.abs(Pi[9] - (pi_hat + r @ Pi)).max() < 1e-13

    pi_hat, r, st, ok = og.push_schedule(9, eps, lam, schedule, hook=hook)
    assert ok and rounds == list(range(1, st.iterations + 1))
    diff = Pi[9] - pi_hat
    assert diff.min() >= -1e-14 and diff.max() <= eps
    deg = np.array([np.count_nonzero(g.edge_u == i) + np.count_nonzero(g.assoc_u == i) for i in range(g.n_u)])
    if schedule == 3:
        assert r.max() <= eps / lam
    elif schedule in (1, 2):
        assert (r <= eps / (og.m_e + og.m_a) * deg + 1e-300).all()


def test_app_s_switches_and_app_never_does():
    """APP(S) reaches the synchronous phase at a small eps; APP and APP(E)
    have no phase switch."""
    g, og, Pi = _small_dense_case()
    lam = og.lambda_thm3()
    assert og.push_schedule(3, 1e-9, lam, 2)[2].switch_iteration > 0
    assert og.push_schedule(3, 1e-9, lam, 1)[2].switch_iteration == -1
    assert og.push_schedule(3, 1e-9, lam, 3)[2].switch_iteration == -1


def test_forward_push_first_push_is_one_step_of_P():
    """Algorithm 2's first push from u leaves alpha at u and (1 - alpha) P[u]
    as residues, with P taken from the dense solve: Pi = alpha (I - (1 -
    alpha) P)^-1, so P = (I - alpha Pi^-1) / (1 - alpha)."""
    g, og, Pi = _small_dense_case()
    P = (np.eye(g.n_u) - O.ALPHA * np.linalg.inv(Pi)) / (1.0 - O.ALPHA)
    seen = []

    def hook(it, pi_hat, r):
        if it == 1:
            seen.append((pi_hat, r))

    og.forward_push(4, 1e-9, max_pushes=1, hook=hook)
    pi_hat, r = seen[0]
    want = np.zeros(g.n_u); want[4] = O.ALPHA
    assert np.abs(pi_hat - want).max() < 1e-15
    assert np.abs(r - (1.0 - O.ALPHA) * P[4]).max() < 1e-12


def test_forward_push_invariant_and_bound():
    """FP keeps Lemma 2 after every single push and stops with every residue
    under r_max (|N(u)| + |A(u)|), which with r_max = eps / (|E| + |E_A|)
    puts it within eps of the exact row; the level-synchronous APP reaches
    the same bound, so the two agree within eps."""
    g, og, Pi = _small_dense_case()
    eps = 1e-6
    r_max = eps / (og.m_e + og.m_a)
    pushes = []

    def hook(it, pi_hat, r):
        pushes.append(it)
        assert np.abs(Pi[2] - (pi_hat + r @ Pi)).max() < 1e-13

    pi_hat, r, st, ok = og.forward_push(2, r_max, max_pushes=200_000, hook=hook)
    assert ok and pushes == list(range(1, st.iterations + 1)) and st.switch_iteration == -1
    deg = np.array([np.count_nonzero(g.edge_u == i) + np.count_nonzero(g.assoc_u == i) for i in range(g.n_u)])
    assert (r <= r_max * deg).all()
    diff = Pi[2] - pi_hat
    assert diff.min() >= -1e-14 and diff.max() <= eps
    app = og.app(2, r_max)[0]
    assert np.abs(app - pi_hat).max() <= eps


def test_forward_push_push_cap():
    g, og, Pi = _small_dense_case()
    _, _, st, ok = og.forward_push(2, 1e-12, max_pushes=3)
    assert not ok and st.iterations == 3


# ---------------------------------------------------------------- lambda

def test_lambda_bounds_column_sums(tiny_oracle, tiny_Pi):
    """Theorem 3: lambda >= max_i sum_j pi(u_j, u_i); pi_T never exceeds the column sums."""
    lam, pt = tiny_oracle.lambda_thm3(return_pi_T=True)
    col = tiny_Pi.sum(axis=0)
    assert lam >= col.max()
    assert (pt <= col + 1e-12).all()
    assert lam - col.max() <= tiny_graph_slack(tiny_oracle)


def tiny_graph_slack(og):
    return og.n_u * (1 - O.ALPHA) ** O.lambda_iterations(og.n_u, O.ALPHA) + 1e-9


@pytest.mark.parametrize("m", [2, 5])
def test_lambda_closed_form_private_attributes(m):
    """Closed form B has doubly stochastic P, so pi_T = (1-(1-a)^T) 1 and
    lambda = 1 + (m-1)(1-a)^T."""
    g = complete_bipartite(m, 3, private_attr=True)
    og = O.OracleGraph.from_graph(g)
    for T in (3, 30):
        lam = og.lambda_thm3(T=T)
        assert lam == pytest.approx(1 + (m - 1) * (1 - O.ALPHA) ** T, abs=1e-13)


# ---------------------------------------------------------------- top-k

def test_topk_bruteforce():
    rng = np.random.default_rng(0)
    pi = rng.integers(0, 5, size=40).astype(np.float64) / 7.0
    for k in (1, 5, 40, 60):
        for ex in (-1, 3):
            ids, vals = O.topk(pi, k, ex)
            cand = [(-pi[i], i) for i in range(40) if pi[i] > 0 and i != ex]
            want = [i for _, i in sorted(cand)[:k]]
            assert ids.tolist() == want
            assert vals.tolist() == [pi[i] for i in want]


def test_check_query_rejects_bad_answers(tiny_oracle, tiny_Pi):
    pi_hat, r, _, _ = tiny_oracle.asrp(5, 1e-6, tiny_oracle.lambda_thm3())
    assert O.check_query(tiny_Pi[5], pi_hat, 1e-6, resid=r).ok
    bad = pi_hat.copy()
    bad[10] += 5e-6
    assert not O.check_query(tiny_Pi[5], bad, 1e-6).ok
    bad = pi_hat.copy()
    bad[10] -= 5e-6
    assert not O.check_query(tiny_Pi[5], bad, 1e-6).ok


# ---------------------------------------------------------------- planted mistakes

def _wrong_PS_swapped_normalisers(g):
    W = O._dense_w(g.n_u, g.n_v, g.edge_u, g.edge_v, g.edge_w)
    d_u, d_v = W.sum(1), W.sum(0)
    return (W / d_v[None, :]) @ (W.T / d_u[None, :])


def test_planted_mistakes_fail_a_pin():
    """Plausible slips in Eq. 1 / Def. 2 / Algorithm 1 each fail one of the pins above."""
    fx = json.load(open(os.path.join(GOLDEN, "example1.json")))
    g = make(fx["n_u"], fx["n_v"], fx["n_attr"], fx["edges"], fx["assoc"])
    # (1) normalisers of Eq. 1 swapped -> rows are no longer stochastic.
    gw = small_weighted(seed=9)
    assert np.abs(_wrong_PS_swapped_normalisers(gw).sum(axis=1) - 1).max() > 1e-3
    # (1b) d(v) replaced by d(u_j) of the target -> Example 1 values change.
    W = O._dense_w(g.n_u, g.n_v, g.edge_u, g.edge_v, g.edge_w)
    d_u = W.sum(1)
    wrong = (W / d_u[:, None]) @ (W.T / d_u[None, :])
    assert wrong[0, 1] != pytest.approx(0.375)
    # (2) beta term dropped -> closed form B changes.
    gb = complete_bipartite(2, 3, private_attr=True)
    P_wrong = O.dense_PS(gb)
    pi_wrong = O.ALPHA * np.linalg.inv(np.eye(2) - (1 - O.ALPHA) * P_wrong)[0]
    assert abs(pi_wrong[0] - 0.6067616) > 1e-3
    # (3) transposed operand (P^T instead of P) -> Perron-vector pin fails.
    gw = small_weighted(seed=9)
    P = O.dense_P(gw)
    pi_t = O.ALPHA * np.linalg.inv(np.eye(gw.n_u) - (1 - O.ALPHA) * P.T)[0]
    pi_ok = O.exact_dense(gw)[0]
    assert np.abs(pi_t - pi_ok).max() > 1e-4
    # (4) restart weight applied as (1-alpha) instead of alpha -> closed form A fails.
    ga = complete_bipartite(4, 3, private_attr=False)
    Pa = O.dense_P(ga)
    pi_bad = (1 - O.ALPHA) * np.linalg.inv(np.eye(4) - O.ALPHA * Pa)[0]
    assert abs(pi_bad[0] - 0.3625) > 1e-3


def test_missing_weights_mean_unit_weights():
    """A weight array left out stands for weight 1 everywhere (C and dense forms)."""
    g = complete_bipartite(3, 2, private_attr=False)
    g0 = types.SimpleNamespace(**{**vars(g), "edge_w": None, "assoc_w": None})
    assert np.array_equal(O.dense_P(g), O.dense_P(g0))
    a, _ = O.OracleGraph.from_graph(g).power_series(1)
    b, _ = O.OracleGraph.from_graph(g0).power_series(1)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- acceptance checks

# Exact scores of a hand-made row (source 0): ranked without the source,
# 1 (0.20) > 2 (0.15) > 4 (0.1000004) > 3 (0.10) > 5 (0.05) > 6 (0.01) > 7 (0).
BAND_PI = np.array([0.5, 0.20, 0.15, 0.10, 0.1000004, 0.05, 0.01, 0.0])


def test_topk_band_accepts_the_exact_list_and_swaps_inside_the_band():
    # k = 3, delta = 1e-6: pi_(3) = 0.1000004, band [0.0999984, 0.1000024]
    # holds nodes 3 and 4, so either may take the third place.
    assert O.topk_band_ok(BAND_PI, np.array([1, 2, 4]), 3, 1e-6, source=0)
    assert O.topk_band_ok(BAND_PI, np.array([1, 2, 3]), 3, 1e-6, source=0)
    assert O.topk_band_ok(BAND_PI, np.array([2, 3, 1]), 3, 1e-6, source=0)
    # A tighter delta puts node 3 below the band.
    assert not O.topk_band_ok(BAND_PI, np.array([1, 2, 3]), 3, 1e-8, source=0)


@pytest.mark.parametrize("ids,why", [
    ([1, 4, 3], "node 2 scores above pi_(k) + 2 delta and is missing"),
    ([1, 2, 5], "node 5 scores below pi_(k) - 2 delta"),
    ([0, 1, 2], "the source is listed"),
    ([1, 2, 4, 3], "more than k ids"),
    ([1, 2, 2], "a repeated id"),
    ([1, 2], "a short list that misses nodes scoring above delta"),
    ([1, 2, 9], "an id outside U"),
])
def test_topk_band_rejects(ids, why):
    assert not O.topk_band_ok(BAND_PI, np.array(ids), 3, 1e-6, source=0), why
    assert not O.check_query(BAND_PI, BAND_PI, 1e-7, k=3, source=0, topk_ids=np.array(ids)).ok, why


def test_topk_band_short_list_when_few_scores_are_positive():
    # Only nodes 1 and 2 score above delta = 0.02 (node 6 scores 0.01 <= delta
    # and may come out as zero); k = 6 then allows the list [1, 2, 4, 3, 5].
    assert O.topk_band_ok(BAND_PI, np.array([1, 2, 4, 3, 5]), 6, 0.02, source=0)
    assert not O.topk_band_ok(BAND_PI, np.array([1, 2, 4, 3]), 6, 1e-6, source=0)


def test_check_query_rejects_a_mass_error(tiny_oracle, tiny_Pi):
    """Lemma 2 (Eq. 5) summed over U: sum pi_hat + sum r = 1 without dangling nodes."""
    pi_hat, r, _, _ = tiny_oracle.asrp(7, 1e-6, tiny_oracle.lambda_thm3())
    chk = O.check_query(tiny_Pi[7], pi_hat, 1e-6, resid=r)
    assert chk.ok and chk.mass_err < 1e-12
    for d in (1e-4, -1e-4):
        bad = r.copy()
        bad[int(np.argmax(r))] += d
        chk = O.check_query(tiny_Pi[7], pi_hat, 1e-6, resid=bad)
        assert not chk.ok and chk.mass_err == pytest.approx(1e-4, rel=1e-6)
