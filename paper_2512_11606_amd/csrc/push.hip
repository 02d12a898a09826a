// Residue push of one AHPP query on gfx950 (Algorithm 4, level-synchronous).
//
// One round of Algorithm 4 (the U loop, then the V loop, then the attribute
// loop of Algorithm 3) is computed as two pull-form gathers over the CSRs
// built at load, plus fix-ups for long rows and a control step:
//
//   k_gather<kBack>  V and attribute rows x:
//       z(x) = inv_b(x) * sum_{u in N(x)} w'(u,x) * [r(u) > theta] r(u)
//     where w'(u,v) = w(u,v)(1-beta)(1-alpha)/d(u) for x = v in V and
//     w'(u,a) = w(u,a) beta(1-alpha)/s(u) for attributes.  This is the U loop
//     (every u above the threshold sends (1-alpha) r(u) split by Eq. 1 / Eq. 2
//     weights) followed by the division of the V / attribute residue by
//     d(v) / t(a) that its push-back uses.  n_p += |N(x)| when r(x) > 0.
//   k_gather<kFwdAcc> U rows u:
//       pushed = r(u) > theta;  pi_hat(u) += pushed ? alpha r(u) : 0;
//       r(u) = (pushed ? 0 : r(u)) + sum_{x in N(u), A(u)} w(u,x) z(x)
//     i.e. the reserve update of the U loop and the V / attribute loops'
//     push-back; n_p += |N(u)| + |A(u)| for pushed u; per-workgroup max r.
//   k_fix<mode>   rows longer than one item: chunk sums added in chunk order.
//   k_control     one workgroup: max_u r(u) and n_p from the partials, then
//                 Algorithm 4's stop rule and phase switch.
//
// The U loop of Algorithm 3 writes only V and attribute residues and the V /
// attribute loops write only U residues, so evaluating each loop on the state
// at its start is exactly the paper's round up to the order of floating-point
// additions.  Each wave takes one schedule item (a pack of short rows, or one
// chunk of a long row), so hub rows are spread over many waves.  No
// floating-point atomics are used: every sum has a fixed order and a query's
// result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;
enum Mode { kBack = 0, kFwdAcc = 1, kFwdLambda = 2 };

struct CsrView {
    const int64_t *__restrict__ off;
    const int32_t *__restrict__ col;
    const float *__restrict__ w;
    const WorkItem *__restrict__ items;
    int64_t n_items;
    const SplitRow *__restrict__ split;
    int64_t n_split;
    const int64_t *__restrict__ item_e0;
    const int32_t *__restrict__ item_ne;
};

CsrView view(const DevCsr &c) {
    return CsrView{c.off, c.col, c.w, c.items, c.n_items, c.split, c.n_split, c.item_e0, c.item_ne};
}

struct GatherArgs {
    CsrView c;
    const float *x;             // gathered vector
    float *y;                   // rows written (z, r or y)
    float *aux;                 // kFwdAcc: pi_hat; kFwdLambda: running sum
    const float *inv_b;         // kBack: row scale
    float *part;                // chunk partial sums (one slot per item)
    const Control *ctl;         // nullable: no early exit, threshold `theta`
    float theta;                // threshold when ctl is null
    float alpha;
    float *blk_f;               // per-workgroup max, nullable
    unsigned long long *blk_u;  // per-workgroup n_p, nullable
    const float *deg;           // |N(u)| + |A(u)| of U nodes (Algorithm 3's thresholds), nullable
};

// Row epilogues: pre(row) is loaded early, with the row's entries;
// full(row, s, pre, len) finishes a row of len entries whose sum is s.
template <int kMode>
struct Epi;

template <>
struct Epi<kBack> {
    float *z;
    const float *inv_b;
    unsigned long long np = 0;
    float mx = 0.0f;
    __device__ float2 pre(int64_t row) const { return make_float2(inv_b[row], 0.0f); }
    __device__ void full(int64_t row, float s, float2 p, int64_t len) {
        const float v = p.x * s;
        z[row] = v;
        if (v > 0.0f) np += (unsigned long long)len;
    }
};

template <>
struct Epi<kFwdAcc> {
    float *r;
    float *pi;
    float theta, alpha;
    // Algorithm 3's per-node thresholds r_max deg(u): for pushing (node) and
    // for the stop rule (ratio: the tracked max is r(u) / (r_max deg(u))).
    bool node = false, ratio = false;
    float r_max = 0.0f;
    const float *deg = nullptr;
    unsigned long long np = 0;
    float mx = 0.0f;
    __device__ float2 pre(int64_t row) const { return make_float2(r[row], pi[row]); }
    __device__ void full(int64_t row, float s, float2 p, int64_t len) {
        const float t_u = (node || ratio) ? r_max * deg[row] : 0.0f;
        const bool pushed = p.x > (node ? t_u : theta);
        if (pushed) {
            pi[row] = p.y + alpha * p.x;
            np += (unsigned long long)len;
        }
        const float v = (pushed ? 0.0f : p.x) + s;
        r[row] = v;
        if (ratio) mx = fmaxf(mx, t_u > 0.0f ? v / t_u : (v > 0.0f ? FLT_MAX : 0.0f));
        else mx = fmaxf(mx, v);
    }
};

// Theorem 3 sweep: acc += alpha y_old; y = s.
template <>
struct Epi<kFwdLambda> {
    float *y;
    float *acc;
    float alpha;
    unsigned long long np = 0;
    float mx = 0.0f;
    __device__ float2 pre(int64_t row) const { return make_float2(y[row], acc[row]); }
    __device__ void full(int64_t row, float s, float2 p, int64_t) {
        acc[row] = p.y + alpha * p.x;
        y[row] = s;
    }
};

template <int kMode>
__device__ __forceinline__ Epi<kMode> make_epi(const GatherArgs &a, float theta) {
    if constexpr (kMode == kBack) {
        return Epi<kBack>{a.y, a.inv_b};
    } else if constexpr (kMode == kFwdAcc) {
        Epi<kFwdAcc> e{a.y, a.aux, theta, a.alpha};
        if (a.ctl) {
            e.node = a.ctl->node_thr != 0;
            e.ratio = a.ctl->stop_ratio != 0;
            e.r_max = a.ctl->r_max;
            e.deg = a.deg;
        }
        return e;
    } else {
        return Epi<kFwdLambda>{a.y, a.aux, a.alpha};
    }
}

// Writes the workgroup's max and n_p to its slots.
template <int kMode>
__device__ __forceinline__ void flush_stat(const GatherArgs &a, Epi<kMode> &e) {
    __shared__ unsigned long long lds[4];
    __shared__ float ldsf[4];
    const unsigned long long v = block_sum<unsigned long long>(e.np, lds);
    const float m = block_max_f(e.mx, ldsf);
    if (threadIdx.x == 0) {
        if (a.blk_u) a.blk_u[blockIdx.x] = v;
        if (a.blk_f) a.blk_f[blockIdx.x] = m;
    }
}

__device__ __forceinline__ float r_max_of(const GatherArgs &a) { return a.ctl ? a.ctl->r_max : 0.0f; }

// Terms of entries e0 + lane + 64 k (k < kPerLane, < ne): w(e) * x(col(e)),
// where the back gather keeps x only above the threshold.  All loads of a
// lane are issued before any is used.
template <bool kUnit, bool kThr, bool kNode>
__device__ __forceinline__ void load_terms(const CsrView &c, const float *__restrict__ x, int64_t e0, int ne,
                                           float theta, const float *__restrict__ deg, float r_max,
                                           float (&t)[kPerLane]) {
    const int lane = threadIdx.x & (kWave - 1);
    int32_t ci[kPerLane];
    float wv[kPerLane];
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
        const int i = lane + k * kWave;
        ci[k] = i < ne ? c.col[e0 + i] : -1;
    }
    if constexpr (!kUnit) {
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int i = lane + k * kWave;
            wv[k] = i < ne ? c.w[e0 + i] : 0.0f;
        }
    }
    float th[kPerLane];
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
        th[k] = theta;
        if constexpr (kNode) th[k] = ci[k] >= 0 ? r_max * deg[ci[k]] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
        float v = ci[k] >= 0 ? x[ci[k]] : 0.0f;
        if constexpr (kThr) v = v > th[k] ? v : 0.0f;
        t[k] = kUnit ? v : v * wv[k];
    }
}

// The wave's share of the schedule (grid-stride over items).  Every load of
// an item that does not depend on another (entries, row bounds, epilogue
// inputs, the next item's descriptor) is issued before the first wait.
template <bool kUnit, int kMode, bool kNode>
__device__ __forceinline__ void spmv_items(const GatherArgs &a, float theta, float *prod, Epi<kMode> &epi) {
    constexpr int kRowsPerLane = kMaxRowsPerItem / kWave;
    constexpr bool kThr = kMode == kBack;
    const CsrView &c = a.c;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    // The next item's descriptor, first entry and count are read a step
    // ahead, so an item's entry loads wait on no other load.
    WorkItem next = WorkItem{0, 0};
    int64_t next_e0 = 0;
    int32_t next_ne = 0;
    if (wave0 < c.n_items) {
        next = c.items[wave0];
        next_e0 = c.item_e0[wave0];
        next_ne = c.item_ne[wave0];
    }
    for (int64_t it = wave0; it < c.n_items; it += stride) {
        const WorkItem item = next;
        const int64_t item_e0 = next_e0;
        const int32_t item_ne = next_ne;
        if (it + stride < c.n_items) {
            next = c.items[it + stride];
            next_e0 = c.item_e0[it + stride];
            next_ne = c.item_ne[it + stride];
        }
        float t[kPerLane];
        if (item.n > 0) {
            const int64_t r0 = item.row;
            const int64_t e0 = item_e0;
            const int ne = item_ne;
            int64_t rb[kRowsPerLane], re[kRowsPerLane];
            float2 pre[kRowsPerLane];
#pragma unroll
            for (int q = 0; q < kRowsPerLane; ++q) {
                const int j = lane + q * kWave;
                rb[q] = re[q] = e0;
                pre[q] = make_float2(0.0f, 0.0f);
                if (j < item.n) {
                    rb[q] = c.off[r0 + j];
                    re[q] = c.off[r0 + j + 1];
                    pre[q] = epi.pre(r0 + j);
                }
            }
            load_terms<kUnit, kThr, kNode>(c, a.x, e0, ne, theta, a.deg, r_max_of(a), t);
#pragma unroll
            for (int k = 0; k < kPerLane; ++k) {
                const int i = lane + k * kWave;
                if (i < ne) prod[i] = t[k];
            }
            wave_lds_sync();
#pragma unroll
            for (int q = 0; q < kRowsPerLane; ++q) {
                const int j = lane + q * kWave;
                if (j < item.n) {
                    const int b0 = (int)(rb[q] - e0), b1 = (int)(re[q] - e0);
                    float s = 0.0f;
#pragma unroll 4
                    for (int e = b0; e < b1; ++e) s += prod[e];
                    epi.full(r0 + j, s, pre[q], b1 - b0);
                }
            }
            wave_lds_sync();
        } else {
            const int64_t row = item.row;
            const int64_t e0 = item_e0;
            const int ne = item_ne < 0 ? -item_ne : item_ne;
            const bool whole = item_ne > 0;  // the row is this one item
            const float2 pre = whole ? epi.pre(row) : make_float2(0.0f, 0.0f);
            load_terms<kUnit, kThr, kNode>(c, a.x, e0, ne, theta, a.deg, r_max_of(a), t);
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < kPerLane; ++k) s += t[k];
            s = wave_sum(s);
            if (lane == 0) {
                if (whole) epi.full(row, s, pre, ne);
                else a.part[it] = s;
            }
        }
    }
}

__device__ __forceinline__ float round_theta(const GatherArgs &a) { return a.ctl ? a.ctl->theta : a.theta; }

template <bool kUnit, int kMode>
__global__ void __launch_bounds__(kBlock) k_gather(GatherArgs a) {
    __shared__ float prod[kWavesPerBlock][kItemEdges];
    if (a.ctl && a.ctl->done) return;
    const float theta = round_theta(a);
    Epi<kMode> epi = make_epi<kMode>(a, theta);
    // The V/attribute gather thresholds each gathered U residue: by theta,
    // or by Algorithm 3's r_max deg(u) while the query's schedule says so.
    if (kMode == kBack && a.ctl && a.ctl->node_thr)
        spmv_items<kUnit, kMode, kMode == kBack>(a, theta, prod[threadIdx.x >> 6], epi);
    else
        spmv_items<kUnit, kMode, false>(a, theta, prod[threadIdx.x >> 6], epi);
    flush_stat<kMode>(a, epi);
}

// Rows cut into chunks: one wave per row adds its chunk sums (fixed order).
template <int kMode>
__global__ void __launch_bounds__(kBlock) k_fix(GatherArgs a) {
    if (a.ctl && a.ctl->done) return;
    const float theta = round_theta(a);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    Epi<kMode> epi = make_epi<kMode>(a, theta);
    for (int64_t i = wave0; i < a.c.n_split; i += stride) {
        const SplitRow sr = a.c.split[i];
        float s = 0.0f;
        for (int ch = lane; ch < sr.nch; ch += kWave) s += a.part[sr.first_item + ch];
        s = wave_sum(s);
        if (lane == 0) epi.full(sr.row, s, epi.pre(sr.row), a.c.off[sr.row + 1] - a.c.off[sr.row]);
    }
    flush_stat<kMode>(a, epi);
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Schedules of Exp-2: 0 ASRP (Algorithm 4), 1 APP (Algorithm 3, r_max =
// eps / (|E| + |E_A|)), 2 APP(S) (APP with Algorithm 4's switch to
// synchronous rounds), 3 APP(E) (APP with Algorithm 4's threshold eps_f and
// stop rule, no switch).
__global__ void k_query_init(Control *ctl, float *r, int32_t source, float eps_f, int32_t max_iters,
                             int32_t schedule, float r_max, const float *deg) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const bool app_thr = schedule == 1 || schedule == 2;
    const float deg_source = deg ? deg[source] : 0.0f;
    r[source] = 1.0f;
    ctl->theta = eps_f;
    ctl->eps_f = eps_f;
    ctl->r_max = r_max;
    ctl->node_thr = app_thr ? 1 : 0;
    ctl->stop_ratio = app_thr ? 1 : 0;
    ctl->sync_switch = (schedule == 0 || schedule == 2) ? 1 : 0;
    ctl->pad0 = 0;
    // The unit residue at the source is above its threshold unless eps is that large.
    const float t0 = app_thr ? r_max * deg_source : eps_f;
    ctl->done = 1.0f > t0 ? 0 : 1;
    ctl->phase = 1;
    ctl->iter = 0;
    ctl->switch_iter = -1;
    ctl->status = ctl->done ? 1 : 0;
    ctl->max_iters = max_iters;
    ctl->n_p = 0;
    ctl->last_max = app_thr ? (t0 > 0.0f ? 1.0f / t0 : FLT_MAX) : 1.0f;
}

// Per-workgroup partial arrays read by k_control.
struct Partials {
    const float *max_a;
    int n_max_a;
    const float *max_b;
    int n_max_b;
    const unsigned long long *np[4];
    int n_np[4];
};

constexpr int kControlThreads = 1024;

// End of a round: max_u r(u), n_p, then Algorithm 4's stop / switch rule.
__global__ void __launch_bounds__(kControlThreads) k_control(Control *ctl, Partials p, Rule rule) {
    __shared__ float ldsf[kControlThreads / kWave];
    __shared__ unsigned long long lds[kControlThreads / kWave];
    if (ctl->done) return;
    float m = 0.0f;
    unsigned long long np = 0;
    // A thread's loads of all six arrays issue before any is used (one
    // round trip to L2, where the gathers just left the partials, instead of
    // one per array); max and integer sums give the same bits in any order.
    int n_all = max(p.n_max_a, p.n_max_b);
#pragma unroll
    for (int k = 0; k < 4; ++k) n_all = max(n_all, p.n_np[k]);
    constexpr int kU = 8;
    for (int i0 = threadIdx.x; i0 < n_all; i0 += kControlThreads * kU) {
        float va[kU], vb[kU];
        unsigned long long vn[4][kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int i = i0 + j * kControlThreads;
            va[j] = i < p.n_max_a ? p.max_a[i] : 0.0f;
            vb[j] = i < p.n_max_b ? p.max_b[i] : 0.0f;
#pragma unroll
            for (int k = 0; k < 4; ++k) vn[k][j] = i < p.n_np[k] ? p.np[k][i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            m = fmaxf(m, fmaxf(va[j], vb[j]));
#pragma unroll
            for (int k = 0; k < 4; ++k) np += vn[k][j];
        }
    }
    m = block_max_n<kControlThreads / kWave>(m, ldsf);
    np = block_sum_u64_n<kControlThreads / kWave>(np, lds);
    if (threadIdx.x != 0) return;
    const unsigned long long n_p = ctl->n_p + np;
    const int iter = ctl->iter + 1;
    // Stop level: eps_f for max r (ASRP, APP(E)), or 1 for the largest
    // r(u) / (r_max deg(u)) (APP, APP(S)).
    const float level = ctl->stop_ratio ? 1.0f : ctl->eps_f;
    ctl->n_p = n_p;
    ctl->iter = iter;
    ctl->last_max = m;
    if (!(m > level)) {
        ctl->done = 1;
        ctl->status = 1;
    } else if (iter >= ctl->max_iters) {
        ctl->done = 1;
        ctl->status = 2;
    } else if (ctl->phase == 1 && ctl->sync_switch) {
        // Budget of Algorithm 4 with the round count of Theorem 1's proof.
        const double t = (double)logf(m / level) * (double)rule.inv_log;
        if ((double)n_p >= rule.budget_scale * (t > 0.0 ? t : 0.0)) {
            ctl->phase = 2;
            ctl->theta = 0.0f;
            ctl->node_thr = 0;
            ctl->switch_iter = iter;
        }
    }
}

__global__ void k_degrees(const int64_t *off, int64_t n, float *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        deg[i] = (float)(off[i + 1] - off[i]);
}

__global__ void k_max_f32(const float *__restrict__ x, int64_t n, float *blk) {
    __shared__ float ldsf[4];
    float m = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, x[i]);
    m = block_max_f(m, ldsf);
    if (threadIdx.x == 0) blk[blockIdx.x] = m;
}

__global__ void k_sum_f64(const float *__restrict__ x, int64_t n, double *blk) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += (double)x[i];
    s = block_sum<double>(s, lds);
    if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

unsigned capped(int64_t n_units, int64_t per_block, int cap) {
    int64_t g = (n_units + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

Rule make_rule(const Graph &g) {
    Rule r;
    r.alpha = (float)g.alpha;
    r.inv_log = (float)(1.0 / std::log(1.0 / (1.0 - g.alpha)));
    r.budget_scale = 2.0 * (double)(g.m_e + g.m_a);
    return r;
}

// Workgroups of the single-query gathers: four times the batched kernels'
// cap, so each wave has fewer items of its latency-bound chain (m1, per
// launch of the back / forward gather: 176 / 153 us at 1x, 172 / 148 at 2x,
// 166 / 145 at 4x, 172 / 144 at 6x, 173 / 158 at 8x).  Their partials are
// sized for it.
inline int single_cap(const Graph &g) { return 4 * g.grid_cap; }

// Launch shapes of one round.
struct Plan {
    unsigned back, back_fix, fwd, fwd_fix;
};

Plan make_plan(const Graph &g) {
    Plan p;
    p.back = g.back.n_items ? capped(g.back.n_items, kWavesPerBlock, single_cap(g)) : 0;
    p.back_fix = g.back.n_split ? capped(g.back.n_split, kWavesPerBlock, single_cap(g)) : 0;
    p.fwd = capped(g.fwd.n_items, kWavesPerBlock, single_cap(g));
    p.fwd_fix = g.fwd.n_split ? capped(g.fwd.n_split, kWavesPerBlock, single_cap(g)) : 0;
    return p;
}

// Launches a gather and its fix-up; the fix-up's partials go single_cap slots
// after the gather's.
template <int kMode>
void launch_gather(Graph &g, bool unit, const GatherArgs &a, unsigned grid, unsigned grid_fix, hipStream_t s,
                   int prof_kind = -1, double prof_bytes = 0.0, double prof_comp = 0.0) {
    if (grid) {
        auto go = [&] {
            if (unit) hipLaunchKernelGGL((k_gather<true, kMode>), dim3(grid), dim3(kBlock), 0, s, a);
            else hipLaunchKernelGGL((k_gather<false, kMode>), dim3(grid), dim3(kBlock), 0, s, a);
        };
        if (prof_kind >= 0) profiled(g.prof, prof_kind, prof_bytes, prof_comp, s, go);
        else go();
    }
    if (grid_fix) {
        GatherArgs b = a;
        if (b.blk_f) b.blk_f += single_cap(g);
        if (b.blk_u) b.blk_u += single_cap(g);
        hipLaunchKernelGGL((k_fix<kMode>), dim3(grid_fix), dim3(kBlock), 0, s, b);
    }
}

__global__ void k_to_input_order(const float *__restrict__ in, const int32_t *__restrict__ u_new, int64_t n,
                                 float *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[u_new[i]];
}

}  // namespace

void to_input_order(const Graph &g, const float *in, float *out, hipStream_t s) {
    if (g.n_u <= 0) return;
    hipLaunchKernelGGL(k_to_input_order, dim3(capped(g.n_u, kBlock, 4096)), dim3(kBlock), 0, s, in,
                       (const int32_t *)g.u_new, g.n_u, out);
    check_hip(hipGetLastError(), "input order");
}

void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f32, dim3(capped(n, kBlock, 4096)), dim3(kBlock), 0, s, p, v, n);
}

namespace {
// Sizes (elements) of the pieces of one query's buffers.
struct QuerySizes {
    size_t n_u, n_z, items, grid_cap;
};
QuerySizes query_sizes(const Graph &g) {
    auto n1 = [](int64_t n) { return (size_t)(n > 0 ? n : 1); };
    return QuerySizes{n1(g.n_u), n1(g.n_v + g.n_a), n1(std::max(g.fwd.n_items, g.back.n_items)),
                      (size_t)single_cap(g)};
}
size_t round_up_256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

void alloc_query_state(Graph &g) {
    if (g.q.r) return;
    const QuerySizes n = query_sizes(g);
    QueryBufs &b = g.q;
    b.r = (float *)dev_alloc(g, n.n_u * 4, "query residues");
    b.pi = (float *)dev_alloc(g, n.n_u * 4, "query reserves");
    b.out = (float *)dev_alloc(g, n.n_u * 4, "query scores in input order");
    b.z = (float *)dev_alloc(g, n.n_z * 4, "query V/attribute residues");
    b.ctl = (Control *)dev_alloc(g, sizeof(Control), "query control");
    b.part = (float *)dev_alloc(g, n.items * 4, "chunk partials");
    b.blk_max = (float *)dev_alloc(g, 2 * n.grid_cap * 4, "workgroup maxima");
    b.blk_np = (unsigned long long *)dev_alloc(g, 4 * n.grid_cap * 8, "workgroup push counts");
    b.sums = (double *)dev_alloc(g, (size_t)kSumBlocks * 8, "residue sums");
    b.tk = nullptr;  // the graph's top-k scratch
}

void free_query_state(QueryBufs &b) {
    for (void *p : {(void *)b.r, (void *)b.pi, (void *)b.out, (void *)b.z, (void *)b.ctl, (void *)b.part,
                    (void *)b.blk_max, (void *)b.blk_np, (void *)b.sums})
        dfree(p);
    b = QueryBufs{};
}

size_t query_bufs_bytes(const Graph &g) {
    const QuerySizes n = query_sizes(g);
    return 3 * round_up_256(n.n_u * 4) + round_up_256(n.n_z * 4) + round_up_256(sizeof(Control)) +
           round_up_256(n.items * 4) + round_up_256(2 * n.grid_cap * 4) + round_up_256(4 * n.grid_cap * 8) +
           round_up_256((size_t)kSumBlocks * 8) + round_up_256(topk_scratch_bytes(1));
}

QueryBufs carve_query_bufs(const Graph &g, void *base) {
    const QuerySizes n = query_sizes(g);
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += round_up_256(bytes);
        return (void *)q;
    };
    QueryBufs b;
    b.r = (float *)take(n.n_u * 4);
    b.pi = (float *)take(n.n_u * 4);
    b.out = (float *)take(n.n_u * 4);
    b.z = (float *)take(n.n_z * 4);
    b.ctl = (Control *)take(sizeof(Control));
    b.part = (float *)take(n.items * 4);
    b.blk_max = (float *)take(2 * n.grid_cap * 4);
    b.blk_np = (unsigned long long *)take(4 * n.grid_cap * 8);
    b.sums = (double *)take((size_t)kSumBlocks * 8);
    b.tk = take(topk_scratch_bytes(1));
    return b;
}

void single_query_init(Graph &g, const QueryBufs &b, int32_t source, float eps_f, int32_t max_iters, hipStream_t s,
                       int32_t schedule, float r_max) {
    if ((schedule == 1 || schedule == 2) && !g.deg_u) {
        g.deg_u = (float *)dev_alloc(g, (size_t)std::max<int64_t>(g.n_u, 1) * 4, "node degrees");
        if (g.single_round_graph) {  // captured with no degree array
            (void)hipGraphExecDestroy(g.single_round_graph);
            g.single_round_graph = nullptr;
        }
        hipLaunchKernelGGL(k_degrees, dim3(capped(g.n_u, kBlock, 4096)), dim3(kBlock), 0, s, g.fwd.off, g.n_u,
                           g.deg_u);
    }
    launch_fill_f32(b.r, 0.0f, g.n_u, s);
    launch_fill_f32(b.pi, 0.0f, g.n_u, s);
    hipLaunchKernelGGL(k_query_init, dim3(1), dim3(64), 0, s, b.ctl, b.r, source, eps_f, max_iters, schedule,
                       r_max, (const float *)g.deg_u);
    check_hip(hipGetLastError(), "query init");
}

void single_query_round(Graph &g, const QueryBufs &b, hipStream_t s, bool timed) {
    const Plan p = make_plan(g);
    const int prof_back = timed ? 0 : -1, prof_fwd = timed ? 1 : -1;
    GatherArgs back{view(g.back), b.r, b.z, nullptr, g.inv_b, b.part, b.ctl, 0.0f, (float)g.alpha,
                    nullptr, b.blk_np, g.deg_u};
    // Algorithmic bytes: CSR entries (column, weight) and gathered residue per
    // entry, offsets and per-row state per row.
    const double wb = g.fwd.w ? 8.0 : 4.0;
    // Compulsory: the CSR once, the gathered vector once, the per-row state.
    launch_gather<kBack>(g, false, back, p.back, p.back_fix, s, prof_back,
                         12.0 * g.back.nnz + 16.0 * g.back.n_rows,
                         8.0 * g.back.nnz + 16.0 * g.back.n_rows + 4.0 * g.n_u);
    GatherArgs fwd{view(g.fwd), b.z, b.r, b.pi, nullptr, b.part, b.ctl, 0.0f, (float)g.alpha,
                   b.blk_max, b.blk_np + 2 * single_cap(g), g.deg_u};
    launch_gather<kFwdAcc>(g, g.unit, fwd, p.fwd, p.fwd_fix, s, prof_fwd,
                           (wb + 4.0) * g.fwd.nnz + 24.0 * g.fwd.n_rows,
                           wb * g.fwd.nnz + 24.0 * g.fwd.n_rows + 4.0 * (g.n_v + g.n_a));
    const int64_t sc = single_cap(g);
    Partials part{b.blk_max, (int)p.fwd, b.blk_max + sc, (int)p.fwd_fix,
                  {b.blk_np, b.blk_np + sc, b.blk_np + 2 * sc, b.blk_np + 3 * sc},
                  {(int)p.back, (int)p.back_fix, (int)p.fwd, (int)p.fwd_fix}};
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kControlThreads), 0, s, b.ctl, part, make_rule(g));
    check_hip(hipGetLastError(), "round launch");
}

void single_query_rounds(Graph &g, const QueryBufs &b, int n, hipStream_t s, bool own) {
    if (!own || !graphs_enabled(g)) {
        for (int i = 0; i < n; ++i) single_query_round(g, b, s, own);
        return;
    }
    if (!g.single_round_graph)
        g.single_round_graph =
            capture_graph(g, "single round capture", [&](hipStream_t cs) { single_query_round(g, g.q, cs); });
    for (int i = 0; i < n; ++i) check_hip(hipGraphLaunch(g.single_round_graph, s), "round graph launch");
}

void single_query_stats(Graph &g, const QueryBufs &b, double *sum_r, hipStream_t s) {
    const unsigned grid = capped(g.n_u, kBlock, kSumBlocks);
    hipLaunchKernelGGL(k_sum_f64, dim3(grid), dim3(kBlock), 0, s, b.r, g.n_u, b.sums);
    double h[kSumBlocks];
    check_hip(hipMemcpyAsync(h, b.sums, grid * sizeof(double), hipMemcpyDeviceToHost, s), "stats D2H");
    check_hip(hipStreamSynchronize(s), "stats");
    double t = 0.0;
    for (unsigned i = 0; i < grid; ++i) t += h[i];
    *sum_r = t;
}

// Theorem 3 (Eq. 6): PI from the all-ones row vector for T rounds,
// pi_T = sum_{l<T} alpha (1-alpha)^l 1 P^l, lambda = max_i pi_T(u_i) + |U| (1-alpha)^T.
// Each sweep is the round above with every U node pushed (threshold -1).
double compute_lambda(Graph &g, int T, hipStream_t s) {
    float *y = g.q.r, *acc = g.q.pi, *z = g.q.z;
    const Plan p = make_plan(g);
    launch_fill_f32(y, 1.0f, g.n_u, s);
    launch_fill_f32(acc, 0.0f, g.n_u, s);
    launch_fill_f32(z, 0.0f, g.n_v + g.n_a, s);
    for (int t = 0; t < T; ++t) {
        GatherArgs back{view(g.back), y, z, nullptr, g.inv_b, g.q.part, nullptr, -1.0f, (float)g.alpha, nullptr,
                        nullptr};
        launch_gather<kBack>(g, false, back, p.back, p.back_fix, s);
        GatherArgs fwd{view(g.fwd), z, y, acc, nullptr, g.q.part, nullptr, -1.0f, (float)g.alpha, nullptr, nullptr};
        launch_gather<kFwdLambda>(g, g.unit, fwd, p.fwd, p.fwd_fix, s);
        check_hip(hipGetLastError(), "lambda launch");
    }
    const unsigned grid = capped(g.n_u, kBlock, g.grid_cap);
    hipLaunchKernelGGL(k_max_f32, dim3(grid), dim3(kBlock), 0, s, acc, g.n_u, g.q.blk_max);
    std::vector<float> h(grid);
    check_hip(hipMemcpyAsync(h.data(), g.q.blk_max, grid * sizeof(float), hipMemcpyDeviceToHost, s), "lambda D2H");
    check_hip(hipStreamSynchronize(s), "lambda");
    float mx = 0.0f;
    for (float v : h) mx = v > mx ? v : mx;
    return (double)mx + (double)g.n_u * std::pow(1.0 - g.alpha, (double)T);
}

}  // namespace ahpp
