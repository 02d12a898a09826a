// Internal declarations of the gfx950 AHPP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace ahpp {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kBlock = 256;          // threads per workgroup (4 waves)
constexpr int kItemEdges = 512;      // CSR entries handled by one wave item
constexpr int kPerLane = kItemEdges / kWave;
constexpr int kShortRow = 64;        // rows up to this length are packed together
constexpr int kMaxRowsPerItem = 256; // rows per packed item
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
    int32_t *col = nullptr;         // nnz
    float *w = nullptr;             // nnz (nullptr when every weight is 1)
    WorkItem *items = nullptr;      // n_items
    int64_t n_items = 0;
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
    float last_max;       // max_i r(u, u_i) after the last completed round
    float pad0;
};

// Constants of the stop/switch rule of one graph.
struct Rule {
    float alpha;
    float inv_log;        // 1 / ln(1 / (1 - alpha))
    double budget_scale;  // 2 (|E| + |E_A|)
};

// Graph held by a handle.
struct Graph {
    int device = 0;
    int n_cu = 256;
    int grid_cap = 2048;            // workgroups of the gather kernels
    int64_t n_u = 0, n_v = 0, n_a = 0, m_e = 0, m_a = 0;
    double alpha = 0.15, beta = 0.35, lambda = 1.0;
    int32_t lambda_iters = 0;
    bool unit = false;              // every weight is 1
    DevCsr fwd;                     // rows U; cols V then attributes (n_v + a)
    DevCsr back;                    // rows V then attributes; cols U (n_u + u for attribute rows)
    float *c_d = nullptr;           // (1-beta)(1-alpha) / d(u), 0 if d(u) = 0
    float *c_s = nullptr;           // beta (1-alpha) / s(u),    0 if s(u) = 0
    float *inv_b = nullptr;         // 1/d(v) for V rows, 1/t(a) for attribute rows
    int64_t dangling_u = 0;
    int64_t device_bytes = 0;
    double load_ms = 0, lambda_ms = 0;
    // Single-query state (allocated at load).
    float *q_r = nullptr, *q_pi = nullptr, *q_rho = nullptr, *q_z = nullptr;
    Control *q_ctl = nullptr;
    float *part_item = nullptr;            // chunk partial sums, max(n_items) slots
    float *blk_max = nullptr;              // per-workgroup maxima, 2 * grid_cap
    unsigned long long *blk_np = nullptr;  // per-workgroup n_p partials, 3 * grid_cap
    // Top-k scratch.
    void *tk_scratch = nullptr;
    size_t tk_scratch_bytes = 0;
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
void *dev_alloc(Graph &g, size_t bytes, const char *what);

// graph_build.hip
void build_graph(Graph &g, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                 const int32_t *aa, const float *aw, hipStream_t s);
void free_graph(Graph &g);

// push.hip
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void alloc_query_state(Graph &g);
void single_query_init(Graph &g, int32_t source, float eps_f, int32_t max_iters, hipStream_t s);
void single_query_round(Graph &g, hipStream_t s);
void single_query_stats(Graph &g, double *sum_r, hipStream_t s);
double compute_lambda(Graph &g, int T, hipStream_t s);

// topk.hip
size_t topk_scratch_bytes(int64_t n_q);
void topk_launch(const float *scores, int64_t n, int64_t stride_q, int64_t n_q, const int32_t *exclude_dev,
                 int32_t exclude_one, int32_t k, int32_t *idx_out, float *val_out, int32_t *n_out, void *scratch,
                 hipStream_t s);

}  // namespace ahpp
