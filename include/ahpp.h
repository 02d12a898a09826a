/*
 * ahpp.h -- C ABI of the MI355X (gfx950) AHPP library.
 *
 * AHPP is the Attribute-augmented Hidden Personalized PageRank of
 * arXiv 2512.11606 (Def. 2, Eq. 3): for a source u in U,
 *     pi(u, .) = sum_{l>=0} alpha (1-alpha)^l e_u P^l,
 *     P = (1-beta) P_S + beta P_A,
 * with P_S the structure transition matrix of Eq. 1 (two hops U->V->U) and
 * P_A the attribute transition matrix of Eq. 2 (two hops U->attribute->U).
 *
 * The library answers the eps-approximate single-source AHPP query of
 * Section 2.3 (Eq. 4): it returns pi_hat(u, .) over U with
 * 0 <= pi(u,i) - pi_hat(u,i) <= eps (Theorem 2), computed by the residue
 * push of Algorithm 4 (ASRP) with lambda from Theorem 3 (Eq. 6), and the
 * k most similar nodes of u (the top-k use of the scores in Section 5).
 *
 * Conventions shared by every call
 *   - ids are 0-based int32; node sets U = [0, n_u), V = [0, n_v),
 *     attributes = [0, n_attr).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the graph's device (e.g. torch tensors on cuda:N).
 *   - The caller owns every buffer it passes.  The library copies what it
 *     needs and never keeps a caller pointer after a call returns.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Device
 *     outputs are written in stream order; a call returns once its results
 *     are complete on that stream unless stated otherwise.
 *   - No C++ exception crosses this boundary.  Every call returns a status;
 *     on failure ahpp_last_error() describes it (per calling thread).
 *   - A graph handle may be used by one thread at a time.
 *
 * Environment (read at each use; results are bitwise the same under every
 * setting but AHPP_HOT_ROWS, which changes the order of some sums and so
 * the rounding, never the guarantee)
 *   AHPP_BATCH_TILES=<n>  tiles of 256 queries the batched engine runs side
 *                         by side (n > 0), over the tuned or default count.
 *   AHPP_GRAPHS=1         batched and single-query rounds replayed from
 *                         captured HIP graphs instead of plain launches.
 *   AHPP_HOT_ROWS=<n>     at load: at most n hot rows (0..128, 0 = none);
 *                         see ahpp_graph_info_t.hot_rows.
 *   AHPP_LOAD_TRACE=1     at load: the time of each build phase on stderr.
 */
#ifndef AHPP_H
#define AHPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ahpp_graph ahpp_graph_t;

typedef enum {
    AHPP_OK = 0,
    AHPP_ERR_INVALID_ARG = -1,   /* bad id, weight, parameter or size          */
    AHPP_ERR_OUT_OF_MEMORY = -2, /* device or host allocation failed            */
    AHPP_ERR_DEVICE = -3,        /* a HIP runtime call failed, or internal error */
    AHPP_ERR_NOT_CONVERGED = -4  /* max_iters rounds ran before the stop rule   */
} ahpp_status_t;

/* Graph description for ahpp_graph_load (all pointers host memory).
 *   Edges E (Section 2.1): n_edges triples (edge_u[e], edge_v[e], edge_w[e])
 *     with edge_u in U, edge_v in V, weight > 0 and finite; edge_w == NULL
 *     means every weight is 1.  Edges are undirected (w(v,u) = w(u,v)).
 *   Node-attribute associations E_A (Section 2.1): n_assoc triples
 *     (assoc_u[e], assoc_a[e], assoc_w[e]), weight > 0 and finite;
 *     assoc_w == NULL means every value is 1.
 *   Repeated pairs are allowed and behave as one pair with the summed weight
 *   (Eq. 1 and Eq. 2 are linear in each weight).
 *   alpha in (0,1): restart probability; beta in [0,1]: attribute-jumping
 *   probability (Def. 2).
 *   lambda > 0 overrides the Theorem 3 estimate; lambda <= 0 asks the library
 *   to compute Eq. 6 with lambda_iters rounds (<= 0: the smallest T with
 *   n_u (1-alpha)^T <= 0.01) and round it up by a factor 1 + 1e-4.
 *   device: HIP device ordinal that will hold the graph.
 *   cache_dir: NULL or "" for none; else a directory where the load keeps the
 *     lambda it computes under the key of the inputs (ahpp_graph_key) and
 *     where a later load with the same key reads it instead of running the
 *     Theorem 3 sweeps.  The library reads and writes only files named
 *     ahpp-<32 hex digits>.lambda there; a missing or unreadable entry, or
 *     one that fails to store, only means lambda is computed. */
typedef struct {
    int64_t n_u, n_v, n_attr;
    int64_t n_edges;
    const int32_t *edge_u, *edge_v;
    const float *edge_w;
    int64_t n_assoc;
    const int32_t *assoc_u, *assoc_a;
    const float *assoc_w;
    double alpha, beta;
    double lambda;
    int32_t lambda_iters;
    int32_t device;
    const char *cache_dir;
} ahpp_graph_desc_t;

typedef struct {
    int64_t n_u, n_v, n_attr, n_edges, n_assoc;  /* as passed to ahpp_graph_load */
    double alpha, beta;
    double lambda;              /* the value eps is divided by (Algorithm 4)   */
    int32_t lambda_iters;       /* rounds used by Theorem 3 (0 if overridden)  */
    int32_t device;
    int64_t dangling_u;         /* U nodes with no edge or no attribute        */
    int64_t device_bytes;       /* device memory held by the graph            */
    double load_ms, lambda_ms;  /* wall time of the build and of Eq. 6 (or of reading it from the cache) */
    uint64_t key[2];            /* ahpp_graph_key of the inputs, computed on the device at load */
    int32_t lambda_cached;      /* 0 no cache dir, 1 lambda read from the cache, 2 computed and stored,
                                   -1 computed, storing failed */
    int32_t hot_rows;           /* V/attribute rows the batched queries sum as a dense product on the
                                   matrix cores: the longest rows of at least 1,024 entries, at most
                                   128 (AHPP_HOT_ROWS=<n> in the environment at load lowers that cap,
                                   0 turns them off); 0 if none, or if their weight block (6 bytes per
                                   row and U node) would exceed a quarter of the device's memory */
} ahpp_graph_info_t;

/* Per-query statistics.  n_push counts edge visits as Algorithm 4 counts n_p
 * (every phase); sync_switch_iter is the round after which the synchronous
 * phase (threshold 0) began, or -1. */
typedef struct {
    int32_t iters;
    int32_t sync_switch_iter;
    int32_t converged;
    int32_t reserved;
    int64_t n_push;
    double max_residual;        /* max_i r(u, u_i) at return                   */
    double sum_residual;        /* sum_i r(u, u_i) at return                   */
    float ms;                   /* device time of the query (or of its batch)  */
    float pad;
} ahpp_stats_t;

/* Builds the graph on the device: the CSR of U -> (V and attributes) and of
 * (V and attributes) -> U, the normalisers d(u), d(v), s(u), t(a) of Eq. 1 and
 * Eq. 2, the push schedules, and lambda (Theorem 3, Eq. 6).  The device
 * numbers nodes by how often the CSRs name them and drops V nodes without an
 * edge; every id the API takes or returns is the caller's.
 * Synchronous.  On success *out owns all device memory of the graph; a
 * failed load frees everything it allocated.
 * Errors: INVALID_ARG (sizes < 0, ids out of range, weights <= 0 or not
 * finite, alpha or beta out of range, out == NULL), OUT_OF_MEMORY, DEVICE. */
ahpp_status_t ahpp_graph_load(const ahpp_graph_desc_t *desc, ahpp_graph_t **out);

/* Fills *info (host). */
ahpp_status_t ahpp_graph_info(const ahpp_graph_t *g, ahpp_graph_info_t *info);

/* The 128-bit key of a graph description (host only, no device needed): a
 * hash of the sizes, of every element of the six COO arrays with its
 * position, of whether each weight array is given, of alpha and beta, and
 * of the Theorem 3 round count the load would use (0 when lambda is given).
 * Any changed id, weight or parameter changes it; it is what ahpp_graph_load
 * computes on the device and files lambda under (cache_dir).  Ids and
 * weights are not validated here.  key: host uint64_t[2].
 * Errors: INVALID_ARG (NULL argument, sizes, NULL arrays with a count > 0,
 * alpha, beta or lambda out of range). */
ahpp_status_t ahpp_graph_key(const ahpp_graph_desc_t *desc, uint64_t *key);

/* Releases the graph and every device buffer it owns.  NULL is ignored. */
void ahpp_graph_free(ahpp_graph_t *g);

/* eps-approximate single-source query (Eq. 4) by Algorithm 4 (ASRP):
 *   eps_f = eps / lambda; rounds with push threshold eps_f until the budget
 *   n_p >= 2(|E| + |E_A|) log_{1/(1-alpha)}(max_i r(u,u_i) / eps_f) is spent,
 *   then rounds with threshold 0, until max_i r(u,u_i) <= eps_f.
 *   source:    node of U.
 *   eps:       > 0.
 *   max_iters: cap on rounds (<= 0: 100000); reaching it returns
 *              AHPP_ERR_NOT_CONVERGED with the outputs of the last round.
 *   pi_out:    device float[n_u] or NULL: pi_hat(source, .).
 *   resid_out: device float[n_u] or NULL: final residues r(source, .).
 *   k:         0 = no top-k, else k >= 1.
 *   topk_idx / topk_val / topk_n: device int32[k] / float[k] / int32[1]:
 *              the k nodes with the largest pi_hat > 0, source excluded,
 *              sorted by score descending then id ascending; *topk_n <= k is
 *              how many were written.  Required when k > 0.
 *   stats:     host or NULL.
 * Blocks the calling thread until the query has finished on hip_stream. */
ahpp_status_t ahpp_query(ahpp_graph_t *g, int32_t source, double eps, int32_t max_iters,
                         float *pi_out, float *resid_out,
                         int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                         ahpp_stats_t *stats, void *hip_stream);

/* ahpp_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, but every per-query buffer
 * lives in a fixed 64 MiB device array that the library holds on each GPU
 * from graph load until the process ends, so the call makes no hipMalloc,
 * hipFree, event or captured graph.
 *   Arguments and outputs as ahpp_query (outputs are the caller's device
 *   buffers, as there); stats->ms is the host wall time of the call.
 *   Limit: the graph's query buffers (about 12 bytes per U node, 4 per V node
 *   and attribute, plus partials; ~15 MB for 1M U nodes) must fit in 64 MiB,
 *   else INVALID_ARG.
 *   Every call on one GPU shares that GPU's array and finds it holding the
 *   last call's contents (the call clears what must start at zero): calls
 *   that overlap on one GPU, from any thread, graph or stream, race. */
ahpp_status_t ahpp_query_noalloc(ahpp_graph_t *g, int32_t source, double eps, int32_t max_iters,
                                 float *pi_out, float *resid_out,
                                 int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                                 ahpp_stats_t *stats, void *hip_stream);

/* The same query under the push schedules the paper compares in Exp-2
 * (the rounds of Algorithm 3 in every case):
 *   0 ASRP    Algorithm 4 (= ahpp_query).
 *   1 APP     Algorithm 3 with r_max = eps / (|E| + |E_A|): u is pushed when
 *             r(u) > r_max (|N(u)| + |A(u)|); stops when no u is.
 *   2 APP(S)  APP plus Algorithm 4's switch to synchronous rounds, with the
 *             budget's logarithm taken of max_u r(u) / (r_max (|N(u)| +
 *             |A(u)|)); stops by APP's rule.
 *   3 APP(E)  APP with Algorithm 4's threshold eps / lambda and stop rule
 *             max r <= eps / lambda, no switch.
 * Arguments, outputs and errors as ahpp_query (INVALID_ARG also for a
 * schedule outside 0..3); for APP and APP(S), stats->max_residual is the
 * largest r(u) / (r_max (|N(u)| + |A(u)|)), which the stop rule brings to
 * <= 1. */
ahpp_status_t ahpp_query_schedule(ahpp_graph_t *g, int32_t source, double eps, int32_t schedule, int32_t max_iters,
                                  float *pi_out, float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val,
                                  int32_t *topk_n, ahpp_stats_t *stats, void *hip_stream);

/* n_q independent queries answered together (Section 5.1 runs queries
 * independently): the rounds of Algorithm 4 for all of them share each pass
 * over the edge lists.  Each query keeps its own eps_f, threshold, phase and
 * stop rule, so every result satisfies the same guarantee as ahpp_query.
 *   sources: host int32[n_q]; eps: host double[n_q] (each > 0).
 *   pi_out:  device float[n_q * n_u] (row q = query q) or NULL.
 *   k, topk_idx (device int32[n_q*k]), topk_val (device float[n_q*k]),
 *   topk_n (device int32[n_q]): as in ahpp_query, row q for query q.
 *   stats: host ahpp_stats_t[n_q] or NULL.
 * n_q = 0 does nothing and returns OK (n_q < 0: INVALID_ARG).
 * Returns NOT_CONVERGED if any query hit max_iters. Blocks until done. */
ahpp_status_t ahpp_query_batch(ahpp_graph_t *g, int32_t n_q, const int32_t *sources, const double *eps,
                               int32_t max_iters, float *pi_out,
                               int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                               ahpp_stats_t *stats, void *hip_stream);

/* Top-k of a device score vector pi (float[n_u]): the k largest entries
 * with pi > 0, `exclude` left out (-1: none), sorted by score descending then
 * id ascending.  Outputs are device pointers as in ahpp_query.
 * Enqueued on hip_stream; returns after enqueueing. */
ahpp_status_t ahpp_topk(const ahpp_graph_t *g, const float *pi, int32_t k, int32_t exclude,
                        int32_t *idx_out, float *val_out, int32_t *n_out, void *hip_stream);

/* Serving engine: queries that arrive over time share the device with
 * continuous batching.  The engine holds `slots` concurrent queries (lanes of
 * 256-query tiles, each with its own residues, reserves, threshold, phase and
 * stop rule, exactly as ahpp_query_batch); a query waits in a host queue
 * until a slot is free, then runs in the same rounds as every other running
 * query, and leaves its slot as soon as its stop rule holds.  Results are the
 * eps-approximate vectors of Eq. 4 (same guarantee as ahpp_query) reduced to
 * their top-k.  One thread at a time per server. */
typedef struct ahpp_server ahpp_server_t;

/* Creates a server on graph g (which must outlive it).
 *   max_device_bytes: budget for per-query device state; slots = 256 * the
 *     number of 256-query tiles that fit (<= 0: a quarter of the free
 *     memory), at least 256.
 *   max_slots: cap on the slots (<= 0: none), rounded up to whole tiles;
 *     fewer slots mean fewer tiles per round, so each round is shorter.
 *   k: top-k size of every result, 1..2048.  max_iters: round cap per query
 *     (<= 0: 100000).  keep_pi: nonzero keeps each finished query's full
 *     vector until its result is read (ahpp_server_results pi_out).
 * Errors: INVALID_ARG, OUT_OF_MEMORY (budget below one tile), DEVICE. */
ahpp_status_t ahpp_server_create(ahpp_graph_t *g, int64_t max_device_bytes, int32_t max_slots, int32_t k,
                                 int32_t max_iters, int32_t keep_pi, ahpp_server_t **out);
void ahpp_server_free(ahpp_server_t *s);

/* Queues one query (host only, no device work): source in U, eps > 0 (Eq. 4);
 * `tag` comes back with its result. */
ahpp_status_t ahpp_server_submit(ahpp_server_t *s, int64_t tag, int32_t source, double eps);

/* One scheduling step on hip_stream: admit queued queries into free slots,
 * run `rounds` rounds of Algorithm 4 for every running query, then collect
 * the queries whose stop rule held (top-k on the device, copied to the host).
 * Blocks until the step is done.  *n_ready (nullable): results waiting. */
ahpp_status_t ahpp_server_step(ahpp_server_t *s, int32_t rounds, int32_t *n_ready, void *hip_stream);

/* Pops up to max_n finished queries in completion order into host arrays:
 * tags[max_n], topk_idx[max_n * k], topk_val[max_n * k], topk_n[max_n],
 * stats[max_n] (nullable; ms = wall time from the step that admitted the
 * query to the end of the step that collected it),
 * pi_out (device float[max_n * n_u], nullable; requires keep_pi).
 * *n_out = number popped. */
ahpp_status_t ahpp_server_results(ahpp_server_t *s, int32_t max_n, int64_t *tags, int32_t *topk_idx,
                                  float *topk_val, int32_t *topk_n, ahpp_stats_t *stats, float *pi_out,
                                  int32_t *n_out, void *hip_stream);

/* Current counts (host pointers, each nullable). */
ahpp_status_t ahpp_server_info(const ahpp_server_t *s, int32_t *slots, int32_t *running, int32_t *queued,
                               int32_t *ready);

/* Low load on the single-query engine.  A tile round moves the state of all
 * 256 lanes of a tile, however few queries run in it, so at low load a
 * query's latency is its rounds times a full tile round.  With solo_max > 0,
 * a step that finds 1..solo_max queries queued and at most solo_max running
 * in the tiles first answers the queued ones one after another with
 * ahpp_query's engine (the same eps guarantee, Theorem 2; results are
 * ahpp_query's, bit for bit), then runs its rounds for the queries in the
 * tiles; otherwise the queue is admitted into the tiles as before, so under
 * load the server batches.  Such a step uses the graph's single-query buffers, so it must not
 * overlap an ahpp_query, ahpp_query_schedule or ahpp_query_mc call on the
 * same graph.
 *   solo_max: 0 (the default: always batch) .. 256.
 * Errors: INVALID_ARG. */
ahpp_status_t ahpp_server_set_solo(ahpp_server_t *s, int32_t solo_max);

/* Monte Carlo estimate of one AHPP row (Section 3.1; Lemma 1): n_walks
 * alpha-hidden walks from `source`; pi(u, x) ~ (walks that stop at x) /
 * n_walks.  Each walk stops at its node with probability alpha, else moves by
 * one step of P (Eq. 1 / Eq. 2, drawn by weight); a walk that must step from
 * a node with no edge (or no attribute) is lost, as the zero row of P loses
 * that mass.  Randomness: SplitMix64 streams keyed by `seed` and the walk
 * index; the counts, and so every output, depend only on the seed.
 *   n_walks: 1 .. 2^32 - 1 (stop counts are 32-bit; no count can exceed
 *            the walks).  pi_out: device float[n_u] (nullable).
 *   k, topk_idx / topk_val / topk_n: as in ahpp_query (device buffers,
 *   source excluded).  stats: host, nullable.
 * Uses the graph's single-query buffers: one call at a time per graph, as
 * for ahpp_query.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
typedef struct {
    int64_t walks;       /* n_walks */
    int64_t lost;        /* walks ended by an empty row of P */
    int64_t truncated;   /* walks cut at 4096 steps (probability (1-alpha)^4096) */
    int64_t steps;       /* steps of P taken by all walks */
    float ms;            /* device time of the call */
    float pad;
} ahpp_mc_stats_t;
ahpp_status_t ahpp_query_mc(ahpp_graph_t *g, int32_t source, int64_t n_walks, uint64_t seed, float *pi_out,
                            int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n, ahpp_mc_stats_t *stats,
                            void *hip_stream);

/* Schedule autotuner of the batched engine (ahpp_query_batch and servers
 * created afterwards).  Times a few rounds for each candidate schedule --
 * tiles of 256 queries in flight (1, 2, 4, ... up to max_tiles; <= 0: as
 * many as fit in a quarter of the free device memory, at most 16) and 1,
 * 2, 4 or 8 times the default workgroups per tile of the gathers -- keeps
 * the one with the least time per tile-round.  A round reads every CSR
 * entry whatever the frontier, so a few rounds measure the steady state.
 * Results do not depend on the schedule (every sum has a fixed order), only
 * the speed does.  AHPP_BATCH_TILES still overrides the tiles in flight.
 * Blocks until done; overwrites the graph's batch state.  *out (nullable):
 * the choice, the candidates timed, and the time per tile-round of the
 * choice and of the untuned schedule with the most tiles.
 * Errors: INVALID_ARG (NULL graph), OUT_OF_MEMORY, DEVICE. */
typedef struct {
    int32_t tiles_in_flight;
    int32_t workgroup_multiplier;
    int32_t candidates;
    int32_t reserved;
    double ms_per_tile_round;
    double default_ms_per_tile_round;
} ahpp_tune_info_t;
ahpp_status_t ahpp_graph_tune(ahpp_graph_t *g, int32_t max_tiles, ahpp_tune_info_t *out, void *hip_stream);

/* Kernel timing (diagnostics, used by the benchmark's roofline figures).
 * While enabled, the library brackets every launch of its gather kernels with
 * HIP events on the launch stream and adds, per kernel kind, the launch
 * count, the summed elapsed time and two byte counts of each launch:
 *   algo_bytes:       the gathered model -- CSR entries and offsets once, one
 *                     residue value per (entry, running query) (4 bytes in the
 *                     single-query path, the 2-byte transport value in the
 *                     batched path), and the per-(row, query) state the
 *                     epilogue reads and writes;
 *   compulsory_bytes: the CSR once, the gathered vector once per running
 *                     query (each of its rows once), and the same per-row
 *                     state: the least a launch can move, so compulsory bytes
 *                     over the launch time never exceed the HBM bandwidth.
 * Kinds: 0 single-query V/attribute gather, 1 single-query U gather,
 *        2 batched V/attribute gather (rows other than the hot rows),
 *        3 batched U gather, 4 batched hot-row pass (the longest V/attribute
 *        rows summed by streaming the U residues once, plus its reduction).
 * ahpp_profile_enable(g, 1) clears the totals and starts; (g, 0) stops.
 * ahpp_profile_read waits for the recorded events and returns the totals
 * (host pointers, each nullable).  Errors: INVALID_ARG (NULL graph or bad
 * kind), DEVICE. */
ahpp_status_t ahpp_profile_enable(ahpp_graph_t *g, int32_t on);
ahpp_status_t ahpp_profile_read(ahpp_graph_t *g, int32_t kind, int64_t *launches, double *total_ms,
                                double *algo_bytes, double *compulsory_bytes);

/* Text of the last error on the calling thread ("" if none). */
const char *ahpp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AHPP_H */
