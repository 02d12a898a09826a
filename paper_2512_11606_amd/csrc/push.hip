// Residue push of one AHPP query on gfx950 (Algorithm 4, level-synchronous).
//
// One round of Algorithm 4 (the U loop, then the V loop, then the attribute
// loop of Algorithm 3) runs as a short chain of kernels over device-resident
// state:
//
//   k_u_push   (U side, elementwise): for every u with r(u) > theta:
//                pi_hat(u) += alpha r(u); rho_d(u) = c_d(u) r(u);
//                rho_s(u) = c_s(u) r(u); r(u) = 0; n_p += |N(u)| + |A(u)|.
//              Other nodes get rho = 0.  (c_d = (1-beta)(1-alpha)/d(u),
//              c_s = beta(1-alpha)/s(u), so rho_d / rho_s are the U->V and
//              U->attribute increments of Algorithm 3 divided by w(u, .).)
//   k_gather<Back>  (V and attribute rows): z(x) = inv_b(x) sum_u w(u,x) rho(u)
//              = r(x)/d(x) for x in V, r(a)/t(a) for attributes;
//              n_p += |N(x)| for every x with r(x) > 0.
//   k_gather<FwdAcc> (U rows): r(u) += sum_{x in N(u), A(u)} w(u,x) z(x), the
//              V->U and attribute->U push-back; per-workgroup max of r.
//   k_fix<...> rows longer than one wave item: their chunk sums are added in
//              chunk order, then the same epilogue runs.
//   k_control  (one workgroup): max_u r(u) and n_p from the per-workgroup
//              partials; the stop and phase-switch rule of Algorithm 4.
//
// The U loop of Algorithm 3 writes only V and attribute residues and the V /
// attribute loops write only U residues, so computing each loop from the
// state at its start is exactly the paper's round, up to the order of
// floating-point additions.  The gathers are pull-form sparse
// matrix-vector products over the CSRs built at load; each wave takes one
// schedule item (a pack of short rows, or one 512-entry chunk of a long row),
// so hub rows are spread over many waves.  No floating-point atomics are
// used: every sum has a fixed order and results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;
enum Mode { kBack = 0, kFwdAcc = 1, kFwdOver = 2 };

struct CsrView {
    const int64_t *__restrict__ off;
    const int32_t *__restrict__ col;
    const float *__restrict__ w;
    const WorkItem *__restrict__ items;
    int64_t n_items;
    const SplitRow *__restrict__ split;
    int64_t n_split;
};

CsrView view(const DevCsr &c) { return CsrView{c.off, c.col, c.w, c.items, c.n_items, c.split, c.n_split}; }

struct GatherArgs {
    CsrView c;
    const float *x;             // gathered vector
    float *y;                   // output rows
    const float *inv_b;         // kBack: row scale
    float *part;                // chunk partial sums (one slot per item)
    const Control *ctl;         // nullable: no early exit
    float *blk_f;               // per-workgroup max (kFwdAcc), nullable
    unsigned long long *blk_u;  // per-workgroup n_p (kBack), nullable
};

// Row epilogues.
template <int kMode>
struct Epi;

template <>
struct Epi<kBack> {
    float *z;
    const float *inv_b;
    const int64_t *off;
    unsigned long long np = 0;
    __device__ void full(int64_t row, float s) {
        const float v = inv_b[row] * s;
        z[row] = v;
        if (v > 0.0f) np += (unsigned long long)(off[row + 1] - off[row]);
    }
};

template <>
struct Epi<kFwdAcc> {
    float *r;
    float mx = 0.0f;
    __device__ void full(int64_t row, float s) {
        const float v = r[row] + s;
        r[row] = v;
        mx = fmaxf(mx, v);
    }
};

template <>
struct Epi<kFwdOver> {
    float *y;
    __device__ void full(int64_t row, float s) { y[row] = s; }
};

template <int kMode>
__device__ __forceinline__ Epi<kMode> make_epi(const GatherArgs &a) {
    if constexpr (kMode == kBack) return Epi<kBack>{a.y, a.inv_b, a.c.off};
    else if constexpr (kMode == kFwdAcc) return Epi<kFwdAcc>{a.y};
    else return Epi<kFwdOver>{a.y};
}

// Writes the workgroup's statistic (max or n_p) to its slot.
template <int kMode>
__device__ __forceinline__ void flush_stat(const GatherArgs &a, Epi<kMode> &e) {
    if constexpr (kMode == kBack) {
        __shared__ unsigned long long lds[4];
        const unsigned long long v = block_sum<unsigned long long>(e.np, lds);
        if (threadIdx.x == 0 && a.blk_u) a.blk_u[blockIdx.x] = v;
    } else if constexpr (kMode == kFwdAcc) {
        __shared__ float ldsf[4];
        const float m = block_max_f(e.mx, ldsf);
        if (threadIdx.x == 0 && a.blk_f) a.blk_f[blockIdx.x] = m;
    }
}

// Terms w(e) * x(col(e)) of entries e0 + lane + 64 k (k < kPerLane, < ne);
// all loads of a lane are issued before any is used.
template <bool kUnit>
__device__ __forceinline__ void load_terms(const CsrView &c, const float *__restrict__ x, int64_t e0, int ne,
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
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
        const float v = ci[k] >= 0 ? x[ci[k]] : 0.0f;
        t[k] = kUnit ? v : v * wv[k];
    }
}

// The wave's share of the schedule (grid-stride over items).
template <bool kUnit, int kMode>
__device__ __forceinline__ void spmv_items(const GatherArgs &a, float *prod, Epi<kMode> &epi) {
    const CsrView &c = a.c;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t it = wave0; it < c.n_items; it += stride) {
        const WorkItem item = c.items[it];
        float t[kPerLane];
        if (item.n > 0) {
            const int64_t r0 = item.row;
            const int64_t e0 = c.off[r0];
            const int ne = (int)(c.off[r0 + item.n] - e0);
            load_terms<kUnit>(c, a.x, e0, ne, t);
#pragma unroll
            for (int k = 0; k < kPerLane; ++k) {
                const int i = lane + k * kWave;
                if (i < ne) prod[i] = t[k];
            }
            wave_lds_sync();
            for (int j = lane; j < item.n; j += kWave) {
                const int b0 = (int)(c.off[r0 + j] - e0), b1 = (int)(c.off[r0 + j + 1] - e0);
                float s = 0.0f;
                for (int e = b0; e < b1; ++e) s += prod[e];
                epi.full(r0 + j, s);
            }
            wave_lds_sync();
        } else {
            const int64_t row = item.row;
            const int64_t rb = c.off[row], re = c.off[row + 1];
            const int64_t e0 = rb + (int64_t)(-item.n) * kItemEdges;
            const int ne = (int)(re - e0 < kItemEdges ? re - e0 : kItemEdges);
            load_terms<kUnit>(c, a.x, e0, ne, t);
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < kPerLane; ++k) s += t[k];
            s = wave_sum(s);
            if (lane == 0) {
                if (re - rb <= kItemEdges) epi.full(row, s);
                else a.part[it] = s;
            }
        }
    }
}

template <bool kUnit, int kMode>
__global__ void __launch_bounds__(kBlock) k_gather(GatherArgs a) {
    __shared__ float prod[kWavesPerBlock][kItemEdges];
    if (a.ctl && a.ctl->done) return;
    Epi<kMode> epi = make_epi<kMode>(a);
    spmv_items<kUnit, kMode>(a, prod[threadIdx.x >> 6], epi);
    flush_stat<kMode>(a, epi);
}

// Rows cut into chunks: one wave per row adds its chunk sums (fixed order).
template <int kMode>
__global__ void __launch_bounds__(kBlock) k_fix(GatherArgs a) {
    if (a.ctl && a.ctl->done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    Epi<kMode> epi = make_epi<kMode>(a);
    for (int64_t i = wave0; i < a.c.n_split; i += stride) {
        const SplitRow sr = a.c.split[i];
        float s = 0.0f;
        for (int ch = lane; ch < sr.nch; ch += kWave) s += a.part[sr.first_item + ch];
        s = wave_sum(s);
        if (lane == 0) epi.full(sr.row, s);
    }
    flush_stat<kMode>(a, epi);
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_query_init(Control *ctl, float *r, int32_t source, float eps_f, int32_t max_iters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    r[source] = 1.0f;
    ctl->theta = eps_f;
    ctl->eps_f = eps_f;
    ctl->done = (1.0f > eps_f) ? 0 : 1;
    ctl->phase = 1;
    ctl->iter = 0;
    ctl->switch_iter = -1;
    ctl->status = ctl->done ? 1 : 0;
    ctl->max_iters = max_iters;
    ctl->n_p = 0;
    ctl->last_max = 1.0f;
}

// U side of a round (see file comment).
__global__ void __launch_bounds__(kBlock) k_u_push(const Control *ctl, float *__restrict__ r, float *__restrict__ pi,
                                                   float *__restrict__ rho, const float *__restrict__ c_d,
                                                   const float *__restrict__ c_s, const int64_t *__restrict__ off,
                                                   int64_t n_u, float alpha, unsigned long long *blk_np) {
    __shared__ unsigned long long lds[4];
    if (ctl->done) return;
    const float theta = ctl->theta;
    unsigned long long np = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_u; j += stride) {
        const float x = r[j];
        float a = 0.0f, b = 0.0f;
        if (x > theta) {
            pi[j] += alpha * x;
            a = c_d[j] * x;
            b = c_s[j] * x;
            r[j] = 0.0f;
            np += (unsigned long long)(off[j + 1] - off[j]);
        }
        rho[j] = a;
        rho[n_u + j] = b;
    }
    np = block_sum<unsigned long long>(np, lds);
    if (threadIdx.x == 0) blk_np[blockIdx.x] = np;
}

// Per-workgroup partial arrays read by k_control.
struct Partials {
    const float *max_a;
    int n_max_a;
    const float *max_b;
    int n_max_b;
    const unsigned long long *np_a;
    int n_np_a;
    const unsigned long long *np_b;
    int n_np_b;
    const unsigned long long *np_c;
    int n_np_c;
};

// End of a round: max_u r(u), n_p, then Algorithm 4's stop / switch rule.
__global__ void __launch_bounds__(kBlock) k_control(Control *ctl, Partials p, Rule rule) {
    __shared__ float ldsf[4];
    __shared__ unsigned long long lds[4];
    if (ctl->done) return;
    float m = 0.0f;
    unsigned long long np = 0;
    for (int i = threadIdx.x; i < p.n_max_a; i += kBlock) m = fmaxf(m, p.max_a[i]);
    for (int i = threadIdx.x; i < p.n_max_b; i += kBlock) m = fmaxf(m, p.max_b[i]);
    for (int i = threadIdx.x; i < p.n_np_a; i += kBlock) np += p.np_a[i];
    for (int i = threadIdx.x; i < p.n_np_b; i += kBlock) np += p.np_b[i];
    for (int i = threadIdx.x; i < p.n_np_c; i += kBlock) np += p.np_c[i];
    m = block_max_f(m, ldsf);
    np = block_sum<unsigned long long>(np, lds);
    if (threadIdx.x != 0) return;
    const unsigned long long n_p = ctl->n_p + np;
    const int iter = ctl->iter + 1;
    const float eps_f = ctl->eps_f;
    ctl->n_p = n_p;
    ctl->iter = iter;
    ctl->last_max = m;
    if (!(m > eps_f)) {
        ctl->done = 1;
        ctl->status = 1;
    } else if (iter >= ctl->max_iters) {
        ctl->done = 1;
        ctl->status = 2;
    } else if (ctl->phase == 1) {
        // Budget of Algorithm 4 with the round count of Theorem 1's proof.
        const double t = (double)logf(m / eps_f) * (double)rule.inv_log;
        if ((double)n_p >= rule.budget_scale * (t > 0.0 ? t : 0.0)) {
            ctl->phase = 2;
            ctl->theta = 0.0f;
            ctl->switch_iter = iter;
        }
    }
}

// Theorem 3 sweep, U side: acc += alpha y; rho = (c_d y, c_s y).
__global__ void k_lambda_u(const float *__restrict__ y, float *__restrict__ acc, float *__restrict__ rho,
                           const float *__restrict__ c_d, const float *__restrict__ c_s, int64_t n_u, float alpha) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_u; j += stride) {
        const float x = y[j];
        acc[j] += alpha * x;
        rho[j] = c_d[j] * x;
        rho[n_u + j] = c_s[j] * x;
    }
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

// Launch shapes of one round.
struct Plan {
    unsigned u, back, back_fix, fwd, fwd_fix;
};

Plan make_plan(const Graph &g) {
    Plan p;
    p.u = capped(g.n_u, kBlock, g.grid_cap);
    p.back = g.back.n_items ? capped(g.back.n_items, kWavesPerBlock, g.grid_cap) : 0;
    p.back_fix = g.back.n_split ? capped(g.back.n_split, kWavesPerBlock, g.grid_cap) : 0;
    p.fwd = capped(g.fwd.n_items, kWavesPerBlock, g.grid_cap);
    p.fwd_fix = g.fwd.n_split ? capped(g.fwd.n_split, kWavesPerBlock, g.grid_cap) : 0;
    return p;
}

template <int kMode>
void launch_gather(const Graph &g, const GatherArgs &a, unsigned grid, unsigned grid_fix, hipStream_t s) {
    if (grid) {
        if (g.unit) hipLaunchKernelGGL((k_gather<true, kMode>), dim3(grid), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_gather<false, kMode>), dim3(grid), dim3(kBlock), 0, s, a);
    }
    if (grid_fix) {
        GatherArgs b = a;
        if (b.blk_f) b.blk_f += g.grid_cap;
        if (b.blk_u) b.blk_u += g.grid_cap;
        hipLaunchKernelGGL((k_fix<kMode>), dim3(grid_fix), dim3(kBlock), 0, s, b);
    }
}

}  // namespace

void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f32, dim3(capped(n, kBlock, 4096)), dim3(kBlock), 0, s, p, v, n);
}

void alloc_query_state(Graph &g) {
    if (g.q_r) return;
    auto n1 = [](int64_t n) { return (size_t)(n > 0 ? n : 1); };
    g.q_r = (float *)dev_alloc(g, n1(g.n_u) * 4, "query residues");
    g.q_pi = (float *)dev_alloc(g, n1(g.n_u) * 4, "query reserves");
    g.q_rho = (float *)dev_alloc(g, n1(2 * g.n_u) * 4, "query push buffer");
    g.q_z = (float *)dev_alloc(g, n1(g.n_v + g.n_a) * 4, "query V/attribute residues");
    g.q_ctl = (Control *)dev_alloc(g, sizeof(Control), "query control");
    g.part_item = (float *)dev_alloc(g, n1(std::max(g.fwd.n_items, g.back.n_items)) * 4, "chunk partials");
    g.blk_max = (float *)dev_alloc(g, (size_t)2 * g.grid_cap * 4, "workgroup maxima");
    g.blk_np = (unsigned long long *)dev_alloc(g, (size_t)3 * g.grid_cap * 8, "workgroup push counts");
}

void single_query_init(Graph &g, int32_t source, float eps_f, int32_t max_iters, hipStream_t s) {
    launch_fill_f32(g.q_r, 0.0f, g.n_u, s);
    launch_fill_f32(g.q_pi, 0.0f, g.n_u, s);
    hipLaunchKernelGGL(k_query_init, dim3(1), dim3(64), 0, s, g.q_ctl, g.q_r, source, eps_f, max_iters);
    check_hip(hipGetLastError(), "query init");
}

void single_query_round(Graph &g, hipStream_t s) {
    const Plan p = make_plan(g);
    hipLaunchKernelGGL(k_u_push, dim3(p.u), dim3(kBlock), 0, s, g.q_ctl, g.q_r, g.q_pi, g.q_rho, g.c_d, g.c_s, g.fwd.off,
                       g.n_u, (float)g.alpha, g.blk_np);
    GatherArgs back{view(g.back), g.q_rho, g.q_z, g.inv_b, g.part_item, g.q_ctl, nullptr, g.blk_np + g.grid_cap};
    launch_gather<kBack>(g, back, p.back, p.back_fix, s);
    GatherArgs fwd{view(g.fwd), g.q_z, g.q_r, nullptr, g.part_item, g.q_ctl, g.blk_max, nullptr};
    launch_gather<kFwdAcc>(g, fwd, p.fwd, p.fwd_fix, s);
    Partials part{g.blk_max, (int)p.fwd, g.blk_max + g.grid_cap, (int)p.fwd_fix,
                  g.blk_np, (int)p.u, g.blk_np + g.grid_cap, (int)p.back, g.blk_np + 2 * g.grid_cap, (int)p.back_fix};
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, s, g.q_ctl, part, make_rule(g));
    check_hip(hipGetLastError(), "round launch");
}

void single_query_stats(Graph &g, double *sum_r, hipStream_t s) {
    const unsigned grid = capped(g.n_u, kBlock, 1024);
    double *d = nullptr;
    check_hip(hipMallocAsync((void **)&d, grid * sizeof(double), s), "stats scratch");
    hipLaunchKernelGGL(k_sum_f64, dim3(grid), dim3(kBlock), 0, s, g.q_r, g.n_u, d);
    std::vector<double> h(grid);
    check_hip(hipMemcpyAsync(h.data(), d, grid * sizeof(double), hipMemcpyDeviceToHost, s), "stats D2H");
    check_hip(hipFreeAsync(d, s), "stats scratch");
    check_hip(hipStreamSynchronize(s), "stats");
    double t = 0.0;
    for (double v : h) t += v;
    *sum_r = t;
}

// Theorem 3 (Eq. 6): PI from the all-ones row vector for T rounds,
// lambda = max_i pi_T(u_i) + |U| (1-alpha)^T.
double compute_lambda(Graph &g, int T, hipStream_t s) {
    float *y = g.q_r, *acc = g.q_pi, *rho = g.q_rho, *z = g.q_z;
    const Plan p = make_plan(g);
    launch_fill_f32(y, 1.0f, g.n_u, s);
    launch_fill_f32(acc, 0.0f, g.n_u, s);
    for (int t = 0; t < T; ++t) {
        hipLaunchKernelGGL(k_lambda_u, dim3(p.u), dim3(kBlock), 0, s, y, acc, rho, g.c_d, g.c_s, g.n_u, (float)g.alpha);
        GatherArgs back{view(g.back), rho, z, g.inv_b, g.part_item, nullptr, nullptr, nullptr};
        launch_gather<kBack>(g, back, p.back, p.back_fix, s);
        if (!p.back) launch_fill_f32(y, 0.0f, g.n_u, s);
        GatherArgs fwd{view(g.fwd), z, y, nullptr, g.part_item, nullptr, nullptr, nullptr};
        if (p.back) launch_gather<kFwdOver>(g, fwd, p.fwd, p.fwd_fix, s);
        check_hip(hipGetLastError(), "lambda launch");
    }
    const unsigned grid = capped(g.n_u, kBlock, g.grid_cap);
    hipLaunchKernelGGL(k_max_f32, dim3(grid), dim3(kBlock), 0, s, acc, g.n_u, g.blk_max);  // grid <= grid_cap
    std::vector<float> h(grid);
    check_hip(hipMemcpyAsync(h.data(), g.blk_max, grid * sizeof(float), hipMemcpyDeviceToHost, s), "lambda D2H");
    check_hip(hipStreamSynchronize(s), "lambda");
    float mx = 0.0f;
    for (float v : h) mx = v > mx ? v : mx;
    return (double)mx + (double)g.n_u * std::pow(1.0 - g.alpha, (double)T);
}

}  // namespace ahpp
