/*
 * CPU oracle for AHPP (test infrastructure only).
 *
 * This file is the plain, slow reference that the HIP library is checked
 * against.  It shares no code with the HIP library: it builds its own
 * adjacency lists from the COO input and computes everything in double
 * precision.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does.
 *
 * Contents
 *   og_build / og_free      adjacency lists N(u), N(v), A(u), A^-1(a) with
 *                           weights and the normalisers d(u), d(v), s(u), t(a)
 *                           (Section 2.1 notation; Eq. 1 and Eq. 2 denominators)
 *   og_power_series         exact AHPP by the power series of Def. 2 / Eq. 3
 *                           (og_power_series_terms: the same, some terms at a time),
 *                           i.e. Algorithm 1 (PI) written as a truncated sum
 *   og_lambda_thm3          lambda of Theorem 3 (Eq. 6): PI from the all-ones
 *                           row vector, max entry plus |U|(1-alpha)^T
 *   og_asrp                 Algorithm 4 (ASRP) in double precision
 *   og_app                  Algorithm 3 (APP) in double precision
 *   og_forward_push         Algorithm 2 (FP): one node at a time, from a
 *                           FIFO queue, in double precision
 *   og_push_schedule        the four push schedules the paper compares in
 *                           Exp-2: ASRP, APP, APP(S), APP(E)
 *   og_asrp_many            og_asrp over a list of sources, one per thread
 *
 * Dangling nodes (no edge, or no attribute) are allowed: the empty sums of
 * Eq. 1 / Eq. 2 are zero, so their rows of P lose mass.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t n_rows;
    int64_t *off;      /* n_rows + 1 */
    int32_t *col;
    double *w;
} og_adj;

typedef struct {
    int64_t n_u, n_v, n_a, m_e, m_a;
    og_adj u2v, v2u, u2a, a2u;
    double *d_u, *d_v, *s_u, *t_a;
} og_graph;

typedef struct {
    int64_t iterations;
    int64_t switch_iteration;   /* -1 when phase 1 never hit its budget */
    int64_t n_push;             /* n_p counted as in Algorithm 4, all phases */
    double max_residual;
    double sum_residual;
} og_stats;

/* Counting sort of (row, col, w) triples into an adjacency list; rows keep
 * the input order of their entries. */
static int adj_build(og_adj *a, int64_t n_rows, int64_t m, const int32_t *row, const int32_t *col,
                     const float *w) {
    a->n_rows = n_rows;
    a->off = (int64_t *)calloc((size_t)n_rows + 1, sizeof(int64_t));
    a->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    a->w = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int64_t *cur = (int64_t *)malloc((size_t)(n_rows + 1) * sizeof(int64_t));
    if (!a->off || !a->col || !a->w || !cur) { free(cur); return -1; }
    for (int64_t e = 0; e < m; ++e) a->off[row[e] + 1]++;
    for (int64_t i = 0; i < n_rows; ++i) a->off[i + 1] += a->off[i];
    memcpy(cur, a->off, (size_t)(n_rows + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) {
        int64_t p = cur[row[e]]++;
        a->col[p] = col[e];
        a->w[p] = w ? (double)w[e] : 1.0;
    }
    free(cur);
    return 0;
}

static void adj_free(og_adj *a) {
    free(a->off);
    free(a->col);
    free(a->w);
}

/* Row sums of an adjacency list: d(x) = sum of w over N(x). */
static double *row_sums(const og_adj *a) {
    double *s = (double *)calloc((size_t)(a->n_rows > 0 ? a->n_rows : 1), sizeof(double));
    for (int64_t i = 0; i < a->n_rows; ++i)
        for (int64_t p = a->off[i]; p < a->off[i + 1]; ++p) s[i] += a->w[p];
    return s;
}

og_graph *og_build(int64_t n_u, int64_t n_v, int64_t n_a, int64_t m_e, const int32_t *eu, const int32_t *ev,
                   const float *ew, int64_t m_a, const int32_t *au, const int32_t *aa, const float *aw) {
    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    g->n_u = n_u; g->n_v = n_v; g->n_a = n_a; g->m_e = m_e; g->m_a = m_a;
    for (int64_t e = 0; e < m_e; ++e)
        if (eu[e] < 0 || eu[e] >= n_u || ev[e] < 0 || ev[e] >= n_v) { free(g); return NULL; }
    for (int64_t e = 0; e < m_a; ++e)
        if (au[e] < 0 || au[e] >= n_u || aa[e] < 0 || aa[e] >= n_a) { free(g); return NULL; }
    if (adj_build(&g->u2v, n_u, m_e, eu, ev, ew) || adj_build(&g->v2u, n_v, m_e, ev, eu, ew) ||
        adj_build(&g->u2a, n_u, m_a, au, aa, aw) || adj_build(&g->a2u, n_a, m_a, aa, au, aw)) {
        free(g);
        return NULL;
    }
    g->d_u = row_sums(&g->u2v);   /* d(u)  = sum_{v in N(u)} w(u,v)          */
    g->d_v = row_sums(&g->v2u);   /* d(v)  = sum_{u in N(v)} w(u,v)          */
    g->s_u = row_sums(&g->u2a);   /* s(u)  = sum_{a in A(u)} w(u,a)   (Eq. 2) */
    g->t_a = row_sums(&g->a2u);   /* t(a)  = sum_{u in A^-1(a)} w(u,a) (Eq. 2) */
    return g;
}

void og_free(og_graph *g) {
    if (!g) return;
    adj_free(&g->u2v); adj_free(&g->v2u); adj_free(&g->u2a); adj_free(&g->a2u);
    free(g->d_u); free(g->d_v); free(g->s_u); free(g->t_a);
    free(g);
}

void og_normalisers(const og_graph *g, double *d_u, double *d_v, double *s_u, double *t_a) {
    if (d_u) memcpy(d_u, g->d_u, (size_t)g->n_u * sizeof(double));
    if (d_v) memcpy(d_v, g->d_v, (size_t)g->n_v * sizeof(double));
    if (s_u) memcpy(s_u, g->s_u, (size_t)g->n_u * sizeof(double));
    if (t_a) memcpy(t_a, g->t_a, (size_t)g->n_a * sizeof(double));
}

/* y_out = y P with P = (1-beta) P_S + beta P_A, row-vector convention
 * (Eq. 1, Eq. 2, Def. 2).  Written as the two-hop sums through V and through
 * the attributes; z_v and z_a are caller-provided scratch. */
static void apply_P(const og_graph *g, double beta, const double *y, double *y_out, double *z_v, double *z_a) {
    const int64_t n_u = g->n_u, n_v = g->n_v, n_a = g->n_a;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n_v; ++v) {
        double s = 0.0;
        for (int64_t p = g->v2u.off[v]; p < g->v2u.off[v + 1]; ++p) {
            int32_t i = g->v2u.col[p];
            s += y[i] * g->v2u.w[p] / g->d_u[i];          /* w(u_i,v)/d(u_i) */
        }
        z_v[v] = s;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n_a; ++a) {
        double s = 0.0;
        for (int64_t p = g->a2u.off[a]; p < g->a2u.off[a + 1]; ++p) {
            int32_t i = g->a2u.col[p];
            s += y[i] * g->a2u.w[p] / g->s_u[i];          /* w(u_i,a)/s(u_i) */
        }
        z_a[a] = s;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t j = 0; j < n_u; ++j) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t p = g->u2v.off[j]; p < g->u2v.off[j + 1]; ++p) {
            int32_t v = g->u2v.col[p];
            s1 += g->u2v.w[p] * z_v[v] / g->d_v[v];       /* w(v,u_j)/d(v) */
        }
        for (int64_t p = g->u2a.off[j]; p < g->u2a.off[j + 1]; ++p) {
            int32_t a = g->u2a.col[p];
            s2 += g->u2a.w[p] * z_a[a] / g->t_a[a];       /* w(u_j,a)/t(a) */
        }
        y_out[j] = (1.0 - beta) * s1 + beta * s2;
    }
}

/* L further terms of the series of Def. 2 from the current term
 * y = (1-alpha)^l e_u P^l: pi += alpha y, then y <- (1-alpha) y P, L times. */
int og_power_series_terms(const og_graph *g, double alpha, double beta, double *y, double *pi, int L,
                          int nthreads) {
    if (!g || !y || !pi || L < 0) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t n_u = g->n_u;
    double *y2 = (double *)calloc((size_t)n_u, sizeof(double));
    double *z_v = (double *)calloc((size_t)(g->n_v + 1), sizeof(double));
    double *z_a = (double *)calloc((size_t)(g->n_a + 1), sizeof(double));
    for (int l = 0; l < L; ++l) {
        for (int64_t j = 0; j < n_u; ++j) pi[j] += alpha * y[j];
        apply_P(g, beta, y, y2, z_v, z_a);
        for (int64_t j = 0; j < n_u; ++j) y[j] = (1.0 - alpha) * y2[j];
    }
    free(y2); free(z_v); free(z_a);
    return 0;
}

/* ||y||_1, summed in index order. */
double og_l1(const double *y, int64_t n) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += fabs(y[j]);
    return s;
}

/* Exact AHPP (Def. 2): pi_u = sum_{l=0}^{T-1} alpha (1-alpha)^l e_u P^l.
 * The dropped tail sum_{l>=T} alpha (1-alpha)^l e_u P^l is entrywise at most
 * ||(1-alpha)^T e_u P^T||_1, returned in *tail_l1 (Section 3.2: the PI error
 * after T rounds is at most (1-alpha)^T). */
int og_power_series(const og_graph *g, double alpha, double beta, int32_t source, int T, double *pi_out,
                    double *tail_l1, int nthreads) {
    if (!g || source < 0 || source >= g->n_u || T < 0) return -1;
    const int64_t n_u = g->n_u;
    double *y = (double *)calloc((size_t)n_u, sizeof(double));
    memset(pi_out, 0, (size_t)n_u * sizeof(double));
    y[source] = 1.0;                       /* (1-alpha)^0 e_u P^0 */
    og_power_series_terms(g, alpha, beta, y, pi_out, T, nthreads);
    if (tail_l1) *tail_l1 = og_l1(y, n_u);
    free(y);
    return 0;
}

/* Theorem 3 / Eq. 6: pi_T = 1 * sum_{l<T} alpha (1-alpha)^l P^l (PI started
 * from the all-ones row vector); lambda = max_i pi_T(u_i) + |U| (1-alpha)^T.
 * Also returns pi_T (nullable) so tests can compare it with exact column sums. */
double og_lambda_thm3(const og_graph *g, double alpha, double beta, int T, double *pi_T_out, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t n_u = g->n_u;
    double *y = (double *)malloc((size_t)n_u * sizeof(double));
    double *y2 = (double *)calloc((size_t)n_u, sizeof(double));
    double *acc = (double *)calloc((size_t)n_u, sizeof(double));
    double *z_v = (double *)calloc((size_t)(g->n_v + 1), sizeof(double));
    double *z_a = (double *)calloc((size_t)(g->n_a + 1), sizeof(double));
    for (int64_t j = 0; j < n_u; ++j) y[j] = 1.0;
    for (int l = 0; l < T; ++l) {
        for (int64_t j = 0; j < n_u; ++j) acc[j] += alpha * y[j];
        apply_P(g, beta, y, y2, z_v, z_a);
        for (int64_t j = 0; j < n_u; ++j) y[j] = (1.0 - alpha) * y2[j];
    }
    double mx = 0.0;
    for (int64_t j = 0; j < n_u; ++j) mx = acc[j] > mx ? acc[j] : mx;
    if (pi_T_out) memcpy(pi_T_out, acc, (size_t)n_u * sizeof(double));
    free(y); free(y2); free(acc); free(z_v); free(z_a);
    return mx + (double)n_u * pow(1.0 - alpha, (double)T);
}

/* State shared by APP and ASRP: reserve over U, residues over U, V and A. */
typedef struct {
    double *pi, *r_u, *r_v, *r_a;
} push_state;

static int state_alloc(const og_graph *g, push_state *s) {
    s->pi = (double *)calloc((size_t)g->n_u, sizeof(double));
    s->r_u = (double *)calloc((size_t)g->n_u, sizeof(double));
    s->r_v = (double *)calloc((size_t)(g->n_v + 1), sizeof(double));
    s->r_a = (double *)calloc((size_t)(g->n_a + 1), sizeof(double));
    return (s->pi && s->r_u && s->r_v && s->r_a) ? 0 : -1;
}

static void state_free(push_state *s) {
    free(s->pi); free(s->r_u); free(s->r_v); free(s->r_a);
}

/* One round of Algorithm 3's body (its for-loops over U, then V, then A).
 * node_threshold(i) is the residue threshold of U node i; U nodes with
 * residue strictly above it push.  Returns the number of edge visits
 * (the n_p increments of Algorithm 4). */
static int64_t push_round(const og_graph *g, double alpha, double beta, push_state *s, const double *thr_u,
                          double thr_scalar) {
    int64_t np = 0;
    /* U -> V and U -> A.  The loop writes only V/A residues, so the set of U
     * nodes above threshold does not change while it runs. */
    for (int64_t i = 0; i < g->n_u; ++i) {
        double th = thr_u ? thr_u[i] : thr_scalar;
        double r = s->r_u[i];
        if (!(r > th)) continue;
        s->pi[i] += alpha * r;
        double rho = (1.0 - alpha) * r;
        for (int64_t p = g->u2v.off[i]; p < g->u2v.off[i + 1]; ++p)
            s->r_v[g->u2v.col[p]] += (1.0 - beta) * g->u2v.w[p] / g->d_u[i] * rho;
        for (int64_t p = g->u2a.off[i]; p < g->u2a.off[i + 1]; ++p)
            s->r_a[g->u2a.col[p]] += beta * g->u2a.w[p] / g->s_u[i] * rho;
        s->r_u[i] = 0.0;
        np += (g->u2v.off[i + 1] - g->u2v.off[i]) + (g->u2a.off[i + 1] - g->u2a.off[i]);
    }
    /* V -> U: every V node with positive residue pushes all of it back. */
    for (int64_t v = 0; v < g->n_v; ++v) {
        double r = s->r_v[v];
        if (!(r > 0.0)) continue;
        for (int64_t p = g->v2u.off[v]; p < g->v2u.off[v + 1]; ++p)
            s->r_u[g->v2u.col[p]] += g->v2u.w[p] / g->d_v[v] * r;
        s->r_v[v] = 0.0;
        np += g->v2u.off[v + 1] - g->v2u.off[v];
    }
    /* A -> U. */
    for (int64_t a = 0; a < g->n_a; ++a) {
        double r = s->r_a[a];
        if (!(r > 0.0)) continue;
        for (int64_t p = g->a2u.off[a]; p < g->a2u.off[a + 1]; ++p)
            s->r_u[g->a2u.col[p]] += g->a2u.w[p] / g->t_a[a] * r;
        s->r_a[a] = 0.0;
        np += g->a2u.off[a + 1] - g->a2u.off[a];
    }
    return np;
}

static double max_u(const og_graph *g, const double *r) {
    double m = 0.0;
    for (int64_t i = 0; i < g->n_u; ++i) m = r[i] > m ? r[i] : m;
    return m;
}

static double sum_u(const og_graph *g, const double *r) {
    double m = 0.0;
    for (int64_t i = 0; i < g->n_u; ++i) m += r[i];
    return m;
}

/* Optional per-iteration hook for invariant tests: called after every
 * completed round with the current reserve and U residues. */
typedef void (*og_round_hook)(int64_t iteration, const double *pi, const double *r_u, void *user);

/* Algorithm 4 (ASRP).
 *   eps_f = eps / lambda.
 *   Phase 1: rounds of Algorithm 3 with threshold eps_f, counting n_p; after
 *   each round, switch to the synchronous phase once
 *       n_p >= 2 (|E| + |E_A|) * log_{1/(1-alpha)}(max_i r(u,u_i) / eps_f)
 *   (the form used in the proof of Theorem 1; the logarithm is clamped at 0).
 *   Phase 2: rounds with threshold 0 (every U node with positive residue).
 *   Both phases run while some U residue exceeds eps_f.
 * Returns 0, or 1 if max_iters rounds did not reach the stopping rule. */
int og_asrp_hooked(const og_graph *g, double alpha, double beta, int32_t source, double eps, double lambda,
                   int64_t max_iters, double *pi_out, double *r_out, og_stats *st, og_round_hook hook, void *user) {
    if (!g || source < 0 || source >= g->n_u || !(eps > 0) || !(lambda > 0)) return -1;
    push_state s;
    if (state_alloc(g, &s)) { state_free(&s); return -1; }
    s.r_u[source] = 1.0;
    const double eps_f = eps / lambda;
    const double m_total = (double)(g->m_e + g->m_a);
    int64_t n_p = 0, it = 0, switch_it = -1;
    int phase = 1, rc = 0;
    double mx = max_u(g, s.r_u);
    while (mx > eps_f) {
        if (it >= max_iters) { rc = 1; break; }
        n_p += push_round(g, alpha, beta, &s, NULL, phase == 1 ? eps_f : 0.0);
        ++it;
        mx = max_u(g, s.r_u);
        if (hook) hook(it, s.pi, s.r_u, user);
        if (phase == 1) {
            double ratio = mx / eps_f;
            double t = ratio > 1.0 ? log(ratio) / log(1.0 / (1.0 - alpha)) : 0.0;
            if ((double)n_p >= 2.0 * m_total * t) { phase = 2; switch_it = it; }
        }
    }
    memcpy(pi_out, s.pi, (size_t)g->n_u * sizeof(double));
    if (r_out) memcpy(r_out, s.r_u, (size_t)g->n_u * sizeof(double));
    if (st) {
        st->iterations = it;
        st->switch_iteration = switch_it;
        st->n_push = n_p;
        st->max_residual = mx;
        st->sum_residual = sum_u(g, s.r_u);
    }
    state_free(&s);
    return rc;
}

int og_asrp(const og_graph *g, double alpha, double beta, int32_t source, double eps, double lambda,
            int64_t max_iters, double *pi_out, double *r_out, og_stats *st) {
    return og_asrp_hooked(g, alpha, beta, source, eps, lambda, max_iters, pi_out, r_out, st, NULL, NULL);
}

/* Algorithm 3 (APP) with residue threshold r_max (|N(u_i)| + |A(u_i)|). */
int og_app(const og_graph *g, double alpha, double beta, int32_t source, double r_max, int64_t max_iters,
           double *pi_out, double *r_out, og_stats *st) {
    if (!g || source < 0 || source >= g->n_u || !(r_max > 0)) return -1;
    push_state s;
    if (state_alloc(g, &s)) { state_free(&s); return -1; }
    double *thr = (double *)malloc((size_t)g->n_u * sizeof(double));
    for (int64_t i = 0; i < g->n_u; ++i)
        thr[i] = r_max * (double)((g->u2v.off[i + 1] - g->u2v.off[i]) + (g->u2a.off[i + 1] - g->u2a.off[i]));
    s.r_u[source] = 1.0;
    int64_t n_p = 0, it = 0;
    int rc = 0;
    for (;;) {
        int any = 0;
        for (int64_t i = 0; i < g->n_u; ++i)
            if (s.r_u[i] > thr[i]) { any = 1; break; }
        if (!any) break;
        if (it >= max_iters) { rc = 1; break; }
        n_p += push_round(g, alpha, beta, &s, thr, 0.0);
        ++it;
    }
    memcpy(pi_out, s.pi, (size_t)g->n_u * sizeof(double));
    if (r_out) memcpy(r_out, s.r_u, (size_t)g->n_u * sizeof(double));
    if (st) {
        st->iterations = it;
        st->switch_iteration = -1;
        st->n_push = n_p;
        st->max_residual = max_u(g, s.r_u);
        st->sum_residual = sum_u(g, s.r_u);
    }
    free(thr);
    state_free(&s);
    return rc;
}

/* Algorithm 2 (FP).  One U node at a time: a FIFO queue holds the nodes
 * whose residue is above r_max (|N(u)| + |A(u)|); a node taken from it (and
 * still above) keeps alpha of its residue as reserve, clears its residue,
 * and hands rho = (1 - alpha) r to its two-hop neighbours, through V with
 * weight (1 - beta) w(u_i, v) w(v, u_j) / (d(u_i) d(v)) and through the
 * attributes with weight beta w(u_i, a) w(u_j, a) / (s(u_i) t(a)).  A node
 * that a push lifts above its threshold joins the queue unless it is in it.
 * Stops when the queue is empty (no node above its threshold).
 * st->iterations counts node pushes, st->n_push the two-hop entries visited
 * (the per-push cost of Lemma 4).  hook, if given, runs after every push.
 * Returns 0, 1 if max_pushes pushes did not empty the queue, or -1. */
int og_forward_push(const og_graph *g, double alpha, double beta, int32_t source, double r_max, int64_t max_pushes,
                    double *pi_out, double *r_out, og_stats *st, og_round_hook hook, void *user) {
    if (!g || source < 0 || source >= g->n_u || !(r_max > 0)) return -1;
    const int64_t n = g->n_u;
    double *pi = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *thr = (double *)malloc((size_t)n * sizeof(double));
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    char *queued = (char *)calloc((size_t)n, 1);
    if (!pi || !r || !thr || !queue || !queued) {
        free(pi); free(r); free(thr); free(queue); free(queued);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i)
        thr[i] = r_max * (double)((g->u2v.off[i + 1] - g->u2v.off[i]) + (g->u2a.off[i + 1] - g->u2a.off[i]));
    r[source] = 1.0;
    int64_t head = 0, count = 0, pushes = 0, visits = 0;
    int rc = 0;
    if (r[source] > thr[source]) { queue[0] = source; queued[source] = 1; count = 1; }
    while (count > 0) {
        const int32_t i = queue[head];
        head = (head + 1) % n;
        --count;
        queued[i] = 0;
        if (!(r[i] > thr[i])) continue;
        if (pushes >= max_pushes) { rc = 1; break; }
        pi[i] += alpha * r[i];
        const double rho = (1.0 - alpha) * r[i];
        r[i] = 0.0;
        for (int64_t p = g->u2v.off[i]; p < g->u2v.off[i + 1]; ++p) {
            const int32_t v = g->u2v.col[p];
            const double c = (1.0 - beta) * g->u2v.w[p] / (g->d_u[i] * g->d_v[v]) * rho;
            for (int64_t q = g->v2u.off[v]; q < g->v2u.off[v + 1]; ++q) {
                const int32_t j = g->v2u.col[q];
                r[j] += c * g->v2u.w[q];
                if (r[j] > thr[j] && !queued[j]) { queue[(head + count) % n] = j; queued[j] = 1; ++count; }
            }
            visits += g->v2u.off[v + 1] - g->v2u.off[v];
        }
        for (int64_t p = g->u2a.off[i]; p < g->u2a.off[i + 1]; ++p) {
            const int32_t a = g->u2a.col[p];
            const double c = beta * g->u2a.w[p] / (g->s_u[i] * g->t_a[a]) * rho;
            for (int64_t q = g->a2u.off[a]; q < g->a2u.off[a + 1]; ++q) {
                const int32_t j = g->a2u.col[q];
                r[j] += c * g->a2u.w[q];
                if (r[j] > thr[j] && !queued[j]) { queue[(head + count) % n] = j; queued[j] = 1; ++count; }
            }
            visits += g->a2u.off[a + 1] - g->a2u.off[a];
        }
        ++pushes;
        if (hook) hook(pushes, pi, r, user);
    }
    memcpy(pi_out, pi, (size_t)n * sizeof(double));
    if (r_out) memcpy(r_out, r, (size_t)n * sizeof(double));
    if (st) {
        st->iterations = pushes;
        st->switch_iteration = -1;
        st->n_push = visits;
        st->max_residual = max_u(g, r);
        st->sum_residual = sum_u(g, r);
    }
    free(pi); free(r); free(thr); free(queue); free(queued);
    return rc;
}

/* The push schedules of Exp-2, in the rounds of Algorithm 3:
 *   0 ASRP    Algorithm 4 (= og_asrp).
 *   1 APP     Algorithm 3 with r_max = eps / (|E| + |E_A|) (= og_app): push
 *             u when r(u) > r_max (|N(u)| + |A(u)|), until no u does.
 *   2 APP(S)  APP plus Algorithm 4's switch to synchronous rounds: after a
 *             round of phase 1, once
 *                 n_p >= 2 (|E| + |E_A|) log_{1/(1-alpha)}(max_u r(u) / thr(u))
 *             (the number of synchronous rounds that bring every residue
 *             under its own threshold, as Algorithm 4's budget does for
 *             eps_f), rounds push every positive residue; the stop rule
 *             stays APP's.
 *   3 APP(E)  APP with Algorithm 4's threshold eps_f = eps / lambda for
 *             every node and its stop rule max_u r(u) <= eps_f, no switch.
 * Nodes with thr(u) = 0 (no edge and no attribute) count as above their
 * threshold whenever r(u) > 0.  Returns 0, 1 (round cap), or -1. */
int og_push_schedule(const og_graph *g, double alpha, double beta, int32_t source, double eps, double lambda,
                     int32_t schedule, int64_t max_iters, double *pi_out, double *r_out, og_stats *st,
                     og_round_hook hook, void *user) {
    if (schedule == 0)
        return og_asrp_hooked(g, alpha, beta, source, eps, lambda, max_iters, pi_out, r_out, st, hook, user);
    if (!g || source < 0 || source >= g->n_u || !(eps > 0) || !(lambda > 0) || schedule < 0 || schedule > 3)
        return -1;
    push_state s;
    if (state_alloc(g, &s)) { state_free(&s); return -1; }
    const double m_total = (double)(g->m_e + g->m_a);
    const double eps_f = eps / lambda, r_max = eps / m_total;
    double *thr = (double *)malloc((size_t)g->n_u * sizeof(double));
    for (int64_t i = 0; i < g->n_u; ++i)
        thr[i] = r_max * (double)((g->u2v.off[i + 1] - g->u2v.off[i]) + (g->u2a.off[i + 1] - g->u2a.off[i]));
    s.r_u[source] = 1.0;
    int64_t n_p = 0, it = 0, switch_it = -1;
    int phase = 1, rc = 0;
    for (;;) {
        /* Stop rule: APP's per-node thresholds, or eps_f for APP(E). */
        double worst = 0.0;  /* max r(u) / thr(u), or max r(u) / eps_f */
        int above = 0;
        for (int64_t i = 0; i < g->n_u; ++i) {
            const double t = schedule == 3 ? eps_f : thr[i];
            if (s.r_u[i] > t) {
                above = 1;
                const double q = t > 0.0 ? s.r_u[i] / t : INFINITY;
                worst = q > worst ? q : worst;
            }
        }
        if (!above) break;
        if (it >= max_iters) { rc = 1; break; }
        if (schedule == 3) n_p += push_round(g, alpha, beta, &s, NULL, eps_f);
        else n_p += push_round(g, alpha, beta, &s, phase == 1 ? thr : NULL, 0.0);
        ++it;
        if (hook) hook(it, s.pi, s.r_u, user);
        if (schedule == 2 && phase == 1) {
            worst = 0.0;
            for (int64_t i = 0; i < g->n_u; ++i)
                if (s.r_u[i] > thr[i]) {
                    const double q = thr[i] > 0.0 ? s.r_u[i] / thr[i] : INFINITY;
                    worst = q > worst ? q : worst;
                }
            const double t = worst > 1.0 ? log(worst) / log(1.0 / (1.0 - alpha)) : 0.0;
            if ((double)n_p >= 2.0 * m_total * t) { phase = 2; switch_it = it; }
        }
    }
    memcpy(pi_out, s.pi, (size_t)g->n_u * sizeof(double));
    if (r_out) memcpy(r_out, s.r_u, (size_t)g->n_u * sizeof(double));
    if (st) {
        st->iterations = it;
        st->switch_iteration = switch_it;
        st->n_push = n_p;
        st->max_residual = max_u(g, s.r_u);
        st->sum_residual = sum_u(g, s.r_u);
    }
    free(thr);
    state_free(&s);
    return rc;
}

/* Runs og_asrp for n_src sources, one source per thread (queries are
 * independent).  pi_out is n_src x n_u row-major (nullable).  Returns the
 * number of queries that failed. */
/* secs (nullable): wall time of each query on its thread. */
int og_asrp_many(const og_graph *g, double alpha, double beta, int32_t n_src, const int32_t *src, double eps,
                 double lambda, int64_t max_iters, int nthreads, double *pi_out, og_stats *st, double *secs) {
    int bad = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int32_t q = 0; q < n_src; ++q) {
        const double t0 = omp_get_wtime();
        double *pi = pi_out ? pi_out + (size_t)q * (size_t)g->n_u
                            : (double *)malloc((size_t)g->n_u * sizeof(double));
        int rc = og_asrp(g, alpha, beta, src[q], eps, lambda, max_iters, pi, NULL, st ? &st[q] : NULL);
        if (rc != 0) bad += 1;
        if (!pi_out) free(pi);
        if (secs) secs[q] = omp_get_wtime() - t0;
    }
    return bad;
}

int og_max_threads(void) { return omp_get_max_threads(); }
