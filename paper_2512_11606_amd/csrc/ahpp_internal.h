// Internal declarations of the gfx950 AHPP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <functional>
#include <string>
#include <vector>

#include "../../include/ahpp.h"

namespace ahpp {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kBlock = 256;          // threads per workgroup (4 waves)
constexpr int kItemEdges = 1024;     // CSR entries handled by one wave item
constexpr int kCsrPad = 32;          // zero entries (column 0, weight 0) after the last CSR entry
constexpr int kPerLane = kItemEdges / kWave;
constexpr int kShortRow = 64;        // rows up to this length are packed together
constexpr int kMaxRowsPerItem = 128; // rows per packed item (a multiple of kWave)
constexpr int kMaxTopK = 2048;       // largest k the device top-k sorts in LDS
constexpr int kBlocksPerCu = 8;      // workgroups per CU of the gather kernels

// One unit of SpMV work for one wave.
//   n > 0 : rows [row, row + n), each at most kShortRow entries, together at
//           most kItemEdges entries ("packed" item, reduced one row per lane);
//   n <= 0: chunk -n of row `row` (entries [off[row] + (-n) * kItemEdges, ...)),
//           reduced by the whole wave.  A row with more than kItemEdges
//           entries has several chunks; each writes its partial sum to the
//           item's slot and a fix-up pass adds the slots in chunk order.
struct WorkItem {
    int32_t row;
    int32_t n;
};

// A row cut into nch chunks whose items are [first_item, first_item + nch).
struct SplitRow {
    int32_t row;
    int32_t first_item;
    int32_t nch;
    int32_t pad;
};

// A CSR matrix in device memory plus its wave schedule.
struct DevCsr {
    int64_t n_rows = 0, nnz = 0;
    int64_t *off = nullptr;         // n_rows + 1
    int32_t *col = nullptr;         // nnz, then kCsrPad zeros
    float *w = nullptr;             // nnz, then kCsrPad zeros (nullptr when every weight is 1)
    WorkItem *items = nullptr;      // n_items
    int64_t n_items = 0;
    // Per item, so a wave need not read the offsets before its entries: the
    // first entry, and the entry count (a pack of rows, or a whole row) or,
    // for a chunk of a row cut into several, minus its entry count.
    int64_t *item_e0 = nullptr;     // n_items
    int32_t *item_ne = nullptr;     // n_items
    SplitRow *split = nullptr;      // rows cut into several chunks
    int64_t n_split = 0;
    int32_t max_row_len = 0;
};

// Per-query control block, resident in device memory.  Written only by the
// control kernel at the end of each round; read by every kernel.
struct Control {
    float theta;          // push threshold of the current round
    float eps_f;          // eps / lambda
    int32_t done;         // 1 once the query stopped
    int32_t phase;        // 1 = threshold eps_f, 2 = synchronous (threshold 0)
    int32_t iter;         // completed rounds
    int32_t switch_iter;  // round after which phase 2 began, -1 if never
    int32_t status;       // 0 running, 1 converged, 2 round cap reached
    int32_t max_iters;
    unsigned long long n_p;  // edge visits (Algorithm 4's n_p, every phase)
    float last_max;       // max_i r(u, u_i) after the last completed round (ratio form: see stop_ratio)
    float r_max;          // Algorithm 3's residue threshold factor, eps / (|E| + |E_A|)
    int32_t node_thr;     // 1: push u when r(u) > r_max deg(u) (APP; APP(S) before its switch)
    int32_t stop_ratio;   // 1: stop when every r(u) <= r_max deg(u); last_max = max r(u) / (r_max deg(u))
    int32_t sync_switch;  // 1: Algorithm 4's switch to threshold 0 (ASRP, APP(S))
    int32_t pad0;
};

// Device buffers of one single-source query: the graph's own (allocated at
// load) or views into caller-free scratch (ahpp_query_noalloc).
struct QueryBufs {
    float *r = nullptr;                    // [n_u] residues (device numbering)
    float *pi = nullptr;                   // [n_u] reserves (device numbering)
    float *z = nullptr;                    // [n_v + n_a] V / attribute residues over their normaliser
    float *out = nullptr;                  // [n_u] a U vector in input order (top-k input when no output is given)
    Control *ctl = nullptr;
    float *part = nullptr;                 // chunk partial sums, max(n_items) slots
    float *blk_max = nullptr;              // per-workgroup maxima, 2 * grid_cap
    unsigned long long *blk_np = nullptr;  // per-workgroup n_p partials, 4 * grid_cap
    double *sums = nullptr;                // per-workgroup residue sums, kSumBlocks
    void *tk = nullptr;                    // top-k scratch of one query (nullable: the graph's)
};
constexpr int kSumBlocks = 1024;           // workgroups of the residue-sum reduction

// Constants of the stop/switch rule of one graph.
struct Rule {
    float alpha;
    float inv_log;        // 1 / ln(1 / (1 - alpha))
    double budget_scale;  // 2 (|E| + |E_A|)
};

// Queries per batch tile: kVec queries per lane of a wave, so a node's row of
// the tile is kTileQ floats (1 KB) and one gather reads one contiguous row.
constexpr int kVec = 4;
constexpr int kTileQ = kWave * kVec;

// Control of one query inside a batch tile (same rule as Control).
struct QueryCtl {
    float theta;          // push threshold; +inf once the query stopped
    float eps_f;
    int32_t done, phase, iter, switch_iter, status, max_iters;
    unsigned long long n_p;
    float last_max;
    int32_t source;       // -1 for an empty lane
    float theta_q;        // threshold the transport rows Q were cut with (the previous round's theta)
    int32_t pad;
};

struct TileCtl {
    QueryCtl q[kTileQ];
    int32_t all_done;     // every lane of the tile stopped
    int32_t pad[15];
};

// Device state of the batched engine: `tiles` tiles of kTileQ queries, each
// stored node-major ([node][kTileQ], one 1 KB row per node).
struct BatchState {
    int tiles = 0;                  // tiles allocated
    int grid_x = 0;                 // workgroups per tile of the gather kernels
    float *r = nullptr;             // [tiles][n_u][kTileQ] residues
    float *pi = nullptr;            // [tiles][n_u][kTileQ] reserves
    uint16_t *q = nullptr;          // [tiles][n_u][kTileQ] bf16 transport of r (what a push moves)
    float *c = nullptr;             // [tiles][n_v + n_a][kTileQ] V / attribute carries (z - zh)
    uint16_t *zh = nullptr;         // [tiles][n_v + n_a][kTileQ] bf16 transport of z = r_V / d(v), r_A / t(a)
    float *part = nullptr;          // [tiles][max(n_items)][kTileQ]
    TileCtl *ctl = nullptr;         // [tiles]
    float *blk_max = nullptr;       // [tiles][2][grid_x][kTileQ]
    unsigned long long *blk_np = nullptr;  // [tiles][5][grid_x][kTileQ]
    float *hot_part = nullptr;      // [tiles][hot chunks][hot rows][kTileQ]
    float *red_max = nullptr;       // [tiles][control slices][kTileQ] partial maxima
    unsigned long long *red_np = nullptr;  // [tiles][control slices][kTileQ] partial n_p
    float *out = nullptr;           // [tiles * kTileQ][n_u] query-major scores for top-k
    double *sums = nullptr;         // [tiles][grid_cap][kTileQ] residue sums
    int64_t live_q = 0;             // queries still running at the last poll
    // One captured round per number of tiles in flight (replayed on the
    // caller's stream); they name this state's buffers, so they go with it.
    std::vector<std::pair<int, hipGraphExec_t>> round_graphs;
    int graphs_gen = 0;             // Graph::plan_gen the captured rounds were made with
};

// Hot rows: the longest rows of the back CSR (the most popular attributes
// and V nodes, a few percent to tens of percent dense over U).  The batched
// engine does not gather them entry by entry: it sums them as a dense
// product on the matrix cores (hot_dense.hip) over fixed chunks of U, then
// adds the chunk partials in chunk order, so each sum has a fixed order and
// results do not depend on the tiles in flight.
constexpr int kHotMax = 128;             // at most this many hot rows (four 32-row MFMA blocks)
constexpr int64_t kHotMinLen = 1024;     // a hot row has at least one full item of entries
// U chunks of the dense hot pass, a fixed property of the graph so that the
// order of its sums (chunk partials added in chunk order) never depends on
// the tiles in flight.  Longer chunks also cut the partials its reduction
// reads (m1, 4-tile batch, pass and reduction per round: 0.80 ms at 512
// chunks, 0.73 at 256, 0.70 at 128, 0.99 at 64).
constexpr int kDenseChunks = 128;
struct HotSet {
    int32_t n = 0;                       // hot rows (0: none, the batch gathers every row)
    int32_t *rows = nullptr;             // [n] back row of hot index h (longest first)
    int32_t *len = nullptr;              // [n] entries of that row
    WorkItem *cold_items = nullptr;      // back schedule without the hot rows
    int64_t n_cold_items = 0;
    SplitRow *cold_split = nullptr;
    int64_t n_cold_split = 0;
    int64_t cold_nnz = 0, cold_rows = 0;
    // w'(u, x_h) split into three bf16 parts in MFMA operand order, dense_ks
    // K-steps of 16 U rows (U padded with zero weights for every chunking).
    uint16_t *w3 = nullptr;
    int64_t dense_ks = 0;
};

// Weighted-draw tables of the Monte Carlo walks (built on first use).
struct McTables {
    int64_t *f_split = nullptr;  // [n_u] first attribute entry of each fwd row
    double *f_cum = nullptr;     // [fwd nnz] prefix sums of raw weights, restarting at the split
    double *b_cum = nullptr;     // [back nnz] prefix sums of raw weights per back row
};
struct McResult {
    int64_t lost, truncated, steps;
};

// Launch timing of the gather kernels (see ahpp_profile_enable).
constexpr int kProfKinds = 5;
struct ProfLaunch {
    int kind;
    hipEvent_t start, stop;
    double bytes;       // gathered-model bytes of the launch
    double compulsory;  // compulsory bytes of the launch
};
struct Profiler {
    bool on = false;
    std::vector<ProfLaunch> pending;
    int64_t launches[kProfKinds] = {};
    double ms[kProfKinds] = {};
    double bytes[kProfKinds] = {};
    double compulsory[kProfKinds] = {};
};
// Records `kind` around the launches issued by f() when profiling is on.
template <class F>
void profiled(Profiler &p, int kind, double bytes, double compulsory, hipStream_t s, F f) {
    if (!p.on) {
        f();
        return;
    }
    ProfLaunch l{kind, nullptr, nullptr, bytes, compulsory};
    if (hipEventCreate(&l.start) != hipSuccess || hipEventCreate(&l.stop) != hipSuccess) {
        f();
        return;
    }
    (void)hipEventRecord(l.start, s);
    f();
    (void)hipEventRecord(l.stop, s);
    p.pending.push_back(l);
}
void profiler_flush(Profiler &p);
void profiler_void_tail(Profiler &p, int kind, int64_t n);

// Graph held by a handle.
struct Graph {
    int device = 0;
    int n_cu = 256;
    int grid_cap = 2048;            // workgroups of the gather kernels
    // n_v counts the V nodes that have an edge: the device structures number
    // only those (n_v_input is the caller's count).
    int64_t n_u = 0, n_v = 0, n_a = 0, m_e = 0, m_a = 0, n_v_input = 0;
    // U numbering of the device structures: u_new[input id] = device id
    // (on the device and in host memory).  Outputs are gathered back to
    // input order through it.
    int32_t *u_new = nullptr;
    std::vector<int32_t> u_new_host;
    double alpha = 0.15, beta = 0.35, lambda = 1.0;
    int32_t lambda_iters = 0;
    bool unit = false;              // every raw weight is 1 (the fwd CSR stores none)
    DevCsr fwd;                     // rows U; cols V then attributes (n_v + a); raw weights
    DevCsr back;                    // rows V then attributes (n_v + a); cols U; weights
                                    // w(u,x) c_d(u) (V rows) or w(u,x) c_s(u) (attribute rows)
    float *inv_b = nullptr;         // 1/d(v) for V rows, 1/t(a) for attribute rows
    float *deg_u = nullptr;         // |N(u)| + |A(u)| as float (Algorithm 3's thresholds; on first use)
    HotSet hot;                     // batched engine: hot back rows and the cold schedule
    McTables mc;                    // Monte Carlo walks
    int64_t dangling_u = 0;
    int64_t device_bytes = 0;
    double load_ms = 0, lambda_ms = 0;
    uint64_t key[2] = {0, 0};       // key of the inputs (prep_cache.hip)
    int32_t lambda_cached = 0;      // 0 no cache, 1 read from the cache, 2 computed and stored, -1 store failed
    // Single-query state (allocated at load).
    QueryBufs q;
    // Batched engine (allocated on first use, grown on demand).
    BatchState batch;
    Profiler prof;
    // Top-k scratch.
    void *tk_scratch = nullptr;
    size_t tk_scratch_bytes = 0;
    // Captured rounds: a library stream to capture on, and the single-query
    // round (its buffers are fixed at load).
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t single_round_graph = nullptr;
    // Batched schedule picked by batch_tune (0: not tuned): tiles in flight
    // and the multiple of the default workgroups per tile of the gathers.
    int tuned_tiles = 0;
    int tuned_wg_mult = 1;
    int plan_gen = 0;               // bumped when the schedule changes (captured rounds go stale)
};

// Error carrying a status code across internal C++ code (never crosses the ABI).
struct Failure {
    int status;
    std::string msg;
};

void check_hip(hipError_t e, const char *what);
inline void dfree(void *p) {
    if (p) (void)hipFree(p);
}

// Device scratch of n elements (none when n is 0) owned by a scope: freed
// when the scope ends, also when a step in it throws (hipFree waits for work
// that may still use it).
template <typename T>
class DevTemp {
  public:
    DevTemp() = default;
    DevTemp(size_t n, const char *what) {
        if (n) check_hip(hipMalloc(reinterpret_cast<void **>(&p_), n * sizeof(T)), what);
    }
    ~DevTemp() { dfree(p_); }
    DevTemp(const DevTemp &) = delete;
    DevTemp &operator=(const DevTemp &) = delete;
    T *get() const { return p_; }

  private:
    T *p_ = nullptr;
};
void *dev_alloc(Graph &g, size_t bytes, const char *what);

// mc.hip: n_walks walks from source; count[x] = walks stopped at x.
void ensure_mc_tables(Graph &g, hipStream_t s);
void free_mc_tables(McTables &t);
McResult mc_walks(Graph &g, int32_t source, int64_t n_walks, uint64_t seed, int max_steps, unsigned *count,
                  hipStream_t s);
// Walk counts (device numbering) to scores in input order.
void mc_scores(const unsigned *count, const int32_t *u_new, int64_t n, int64_t n_walks, float *out, hipStream_t s);

// prep_cache.hip: the 128-bit key of a graph's inputs (sizes, the six COO
// arrays, alpha, beta, the Theorem 3 round count; the same value on the
// device, over the uploaded arrays, and on the host), and the cache of
// lambda (Eq. 6) under that key in a directory.
struct KeyInput {
    int64_t n_u, n_v, n_attr, n_edges, n_assoc;
    bool has_ew, has_aw;
    double alpha, beta;
    int32_t lambda_iters;
};
void coo_key_device(const KeyInput &in, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                    const int32_t *aa, const float *aw, uint64_t key[2], hipStream_t s);
void coo_key_host(const KeyInput &in, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                  const int32_t *aa, const float *aw, uint64_t key[2]);
bool lambda_cache_read(const std::string &dir, const KeyInput &in, const uint64_t key[2], double *lambda);
bool lambda_cache_write(const std::string &dir, const KeyInput &in, const uint64_t key[2], double lambda);

// hot_dense.hip: the hot rows as a dense MFMA product; the chunking of U
// (kc rows per chunk), its weights' bytes, their build at load, and the
// launch of a batched round (partials [n_chunks][n_hot][kTileQ] per tile,
// added by the hot reduction).
void dense_chunking(int64_t n_u, int64_t *kc, int64_t *n_chunks);
size_t hot_dense_bytes(const Graph &g);
void build_hot_dense(Graph &g, hipStream_t s);
void launch_hot_dense(const Graph &g, const uint16_t *q, int64_t q_stride, const TileCtl *ctl, int nt, float *part,
                      int64_t part_stride, hipStream_t s);

// graph_build.hip (also computes g.key on the device from the uploaded COO)
void build_graph(Graph &g, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                 const int32_t *aa, const float *aw, const KeyInput &kin, hipStream_t s);
void free_graph(Graph &g);

// push.hip
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void alloc_query_state(Graph &g);
void free_query_state(QueryBufs &b);
// Bytes of one query's buffers laid out by carve_query_bufs (256-byte
// aligned pieces), and the buffers carved from `base`.
size_t query_bufs_bytes(const Graph &g);
QueryBufs carve_query_bufs(const Graph &g, void *base);
// out[i] = in[u_new[i]]: a U vector of the device numbering in input order.
void to_input_order(const Graph &g, const float *in, float *out, hipStream_t s);
// schedule: 0 ASRP, 1 APP, 2 APP(S), 3 APP(E) (Exp-2); r_max = eps / (|E| + |E_A|).
void single_query_init(Graph &g, const QueryBufs &b, int32_t source, float eps_f, int32_t max_iters, hipStream_t s,
                       int32_t schedule = 0, float r_max = 0.0f);
// One round; `timed` lets the launch profiler time it (when it is on).
void single_query_round(Graph &g, const QueryBufs &b, hipStream_t s, bool timed = true);
// n rounds.  `own`: b is the graph's own buffers, so the rounds may be
// replayed from a captured HIP graph (which names them) and timed by the
// launch profiler; otherwise every round is plain launches, untimed.
void single_query_rounds(Graph &g, const QueryBufs &b, int n, hipStream_t s, bool own);
bool graphs_enabled(const Graph &g);
hipGraphExec_t capture_graph(Graph &g, const char *what, const std::function<void(hipStream_t)> &record);
void single_query_stats(Graph &g, const QueryBufs &b, double *sum_r, hipStream_t s);
double compute_lambda(Graph &g, int T, hipStream_t s);

// noalloc.hip: a file-scope device array of kNoallocScratchBytes per GPU for
// ahpp_query_noalloc.  noalloc_setup (at graph load, with `device` current)
// looks up its device address once per device; noalloc_scratch returns it
// (nullptr before set-up).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
void noalloc_setup(int device);
void *noalloc_scratch(int device);

// capi.hip: the body of a single-source query on buffers b (see
// single_query_rounds for `own`; with own == false nothing is allocated and
// no event, captured graph or profiler record is made, and stats->ms is the
// host wall time of the call).  Returns the control status (1 converged).
int32_t run_query(Graph &g, const QueryBufs &b, bool own, int32_t source, double eps, int32_t schedule,
                  int32_t max_iters, float *pi_out, float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val,
                  int32_t *topk_n, ahpp_stats_t *stats, hipStream_t s);

// batch.hip
struct AdmitReq {
    int32_t tile, lane, source;
    float eps_f;
};
// Device bytes of one tile (with or without the query-major score buffer).
int64_t batch_tile_bytes(const Graph &g, bool with_out);
void ensure_batch_state(Graph &g, BatchState &b, int tiles, bool with_out);
void free_batch_state(BatchState &b);
// Initialises tiles [0, nt): lane q of tile t gets query t * kTileQ + q
// (sources / eps_f host arrays of n_q entries; lanes beyond n_q are empty).
void batch_init(Graph &g, BatchState &b, int nt, const int32_t *sources, const float *eps_f, int64_t n_q,
                int32_t max_iters, hipStream_t s);
void batch_round(Graph &g, BatchState &b, int nt, hipStream_t s);
// `n` rounds of tiles [0, nt): plain launches, or with AHPP_GRAPHS=1 one
// captured round replayed n times (HIP graphs; never while profiling).
void batch_rounds(Graph &g, BatchState &b, int nt, int n, hipStream_t s);
// Times rounds for each candidate schedule (tiles in flight up to max_tiles,
// workgroups per tile x1, x2, x4) and keeps the fastest per tile-round in g.
struct TuneResult {
    int tiles, wg_mult, candidates;
    double ms_per_tile_round, default_ms_per_tile_round;
};
TuneResult batch_tune(Graph &g, int max_tiles, hipStream_t s);
// Copies tile scores to query-major rows: out[(t*kTileQ + q) * n_u + u] for
// the first n_rows rows.
void batch_scores(Graph &g, BatchState &b, int nt, int64_t n_rows, float *out, hipStream_t s);
// Per-lane residue sums of tiles [t0, t0 + nt) into host sums[(t-t0)*kTileQ + q].
void batch_resid_sums(Graph &g, BatchState &b, int t0, int nt, double *sums, hipStream_t s);
// Serving: all lanes empty; admit queries into lanes (clears their columns);
// copy selected lanes of one tile to query-major rows.
void batch_empty(Graph &g, BatchState &b, int nt, hipStream_t s);
void batch_admit(Graph &g, BatchState &b, const std::vector<AdmitReq> &reqs, int32_t max_iters, hipStream_t s);
void batch_lanes_out(Graph &g, BatchState &b, int tile, const int32_t *d_lanes, int n_sel, float *out,
                     hipStream_t s);

// serve.hip: continuous batching over the lanes of a private batch state.
class Server {
  public:
    Server(Graph &g, int64_t max_device_bytes, int32_t max_slots, int32_t k, int32_t max_iters, bool keep_pi);
    ~Server();
    void submit(int64_t tag, int32_t source, double eps);
    int step(int rounds, hipStream_t s);
    int results(int max_n, int64_t *tags, int32_t *topk_idx, float *topk_val, int32_t *topk_n, ahpp_stats_t *stats,
                float *pi_out, hipStream_t s);
    void info(int32_t *slots, int32_t *running, int32_t *queued, int32_t *ready) const;
    void set_solo(int32_t solo_max) { solo_max_ = solo_max; }
    Graph &graph() { return g_; }

  private:
    struct Pending {
        int64_t tag;
        int32_t source;
        double eps;
    };
    struct Lane {
        bool busy = false;
        int64_t tag = 0;
        int32_t source = -1;
        double t_admit = 0.0;
    };
    struct Result {
        int64_t tag;
        std::vector<int32_t> idx;
        std::vector<float> val;
        ahpp_stats_t st;
        float *d_pi;
    };
    // Answers every queued query on the single-query path (see step).
    void serve_solo(double t_step, hipStream_t s);
    Graph &g_;
    BatchState b_;
    int32_t k_, max_iters_;
    bool keep_pi_;
    int32_t solo_max_ = 0;
    std::vector<Lane> lanes_;
    std::deque<Pending> queue_;
    std::deque<Result> ready_;
    float *d_scores_ = nullptr;     // [kTileQ][n_u]
    int32_t *d_sel_ = nullptr;      // [2][kTileQ]: lanes, then sources
    int32_t *d_idx_ = nullptr;      // [kTileQ][k]
    float *d_val_ = nullptr;        // [kTileQ][k]
    int32_t *d_n_ = nullptr;        // [kTileQ]
    void *d_tk_ = nullptr;
    int64_t own_bytes_ = 0;
};

// topk.hip
size_t topk_scratch_bytes(int64_t n_q);
void topk_launch(const float *scores, int64_t n, int64_t stride_q, int64_t n_q, const int32_t *exclude_dev,
                 int32_t exclude_one, int32_t k, int32_t *idx_out, float *val_out, int32_t *n_out, void *scratch,
                 hipStream_t s);

}  // namespace ahpp
