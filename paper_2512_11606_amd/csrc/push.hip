// Residue push of one AHPP query on gfx950 (Algorithm 4, level-synchronous).
//
// One round of Algorithm 4 (the U loop, then the V loop, then the attribute
// loop of Algorithm 3) is three kernels over device-resident state:
//
//   k_u_push   (U side, elementwise): for every u with r(u) > theta:
//                pi_hat(u) += alpha r(u); rho_d(u) = c_d(u) r(u);
//                rho_s(u) = c_s(u) r(u); r(u) = 0; n_p += |N(u)| + |A(u)|.
//              Other nodes get rho = 0.  (c_d = (1-beta)(1-alpha)/d(u),
//              c_s = beta(1-alpha)/s(u), so rho_d/rho_s are the U->V and
//              U->attribute increments of Algorithm 3 divided by w(u,.).)
//   k_back     (V and attribute rows): z(x) = inv_b(x) * sum_{u} w(u,x) rho(u)
//              = r(x) / d(x) for x in V, r(a) / t(a) for attributes;
//              n_p += |N(x)| for every x with r(x) > 0.
//   k_fwd      (U rows): r(u) += sum_{x in N(u) and A(u)} w(u,x) z(x), i.e. the
//              V->U and attribute->U push-back; max_u r(u) is reduced and the
//              last workgroup applies the stop / switch rule of Algorithm 4.
//
// The U loop of Algorithm 3 writes only V and attribute residues and the V /
// attribute loops write only U residues, so a round computed this way (every
// push of a loop reading the state at the loop's start) is exactly the
// paper's round up to the order of floating-point additions.  The gathers
// are pull-form sparse matrix-vector products over the CSRs built at load;
// each wave takes one schedule item (a pack of short rows, or one chunk of a
// long row), so hub rows are spread over many waves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

struct CsrView {
    const int64_t *__restrict__ off;
    const int32_t *__restrict__ col;
    const float *__restrict__ w;
    const WorkItem *__restrict__ items;
    int64_t n_items;
    uint32_t *split_cnt;
};

CsrView view(const DevCsr &c) { return CsrView{c.off, c.col, c.w, c.items, c.n_items, c.split_cnt}; }

template <bool kUnit>
__device__ __forceinline__ float term(const CsrView &c, const float *__restrict__ x, int64_t e) {
    float v = x[c.col[e]];
    return kUnit ? v : v * c.w[e];
}

// Runs the wave's share of the schedule.  Epi receives complete row sums
// (full) and partial sums of rows cut into nch chunks (partial).
template <bool kUnit, class Epi>
__device__ __forceinline__ void spmv_items(const CsrView &c, const float *__restrict__ x, float *prod, Epi &epi) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t it = wave0; it < c.n_items; it += stride) {
        const WorkItem item = c.items[it];
        if (item.n > 0) {
            const int64_t r0 = item.row;
            const int64_t e0 = c.off[r0];
            const int ne = (int)(c.off[r0 + item.n] - e0);
            for (int i = lane; i < ne; i += kWave) prod[i] = term<kUnit>(c, x, e0 + i);
            wave_lds_sync();
            for (int j = lane; j < item.n; j += kWave) {
                const int a = (int)(c.off[r0 + j] - e0), b = (int)(c.off[r0 + j + 1] - e0);
                float s = 0.0f;
                for (int e = a; e < b; ++e) s += prod[e];
                epi.full(r0 + j, s);
            }
            wave_lds_sync();
        } else {
            const int64_t row = item.row;
            const int64_t rb = c.off[row], re = c.off[row + 1];
            const int64_t e0 = rb + (int64_t)(-item.n) * kItemEdges;
            const int64_t e1 = e0 + kItemEdges < re ? e0 + kItemEdges : re;
            float s = 0.0f;
            for (int64_t e = e0 + lane; e < e1; e += kWave) s += term<kUnit>(c, x, e);
            s = wave_sum(s);
            const int nch = (int)((re - rb + kItemEdges - 1) / kItemEdges);
            if (lane == 0) {
                if (nch == 1) epi.full(row, s);
                else epi.partial(row, s, nch, c.split_cnt);
            }
        }
    }
}

// r(u) += s; tracks the max of the new residues.
struct EpiAccumulate {
    float *r;
    float mx = 0.0f;
    __device__ void full(int64_t row, float s) {
        const float v = r[row] + s;
        r[row] = v;
        mx = fmaxf(mx, v);
    }
    __device__ void partial(int64_t row, float s, int nch, uint32_t *cnt) {
        atomicAdd(&r[row], s);
        __threadfence();
        if (atomicAdd(&cnt[row], 1u) == (uint32_t)(nch - 1)) {
            cnt[row] = 0;
            mx = fmaxf(mx, atomicAdd(&r[row], 0.0f));
        }
    }
};

// y(row) = s (split rows must be zero beforehand).
struct EpiOverwrite {
    float *y;
    __device__ void full(int64_t row, float s) { y[row] = s; }
    __device__ void partial(int64_t row, float s, int nch, uint32_t *cnt) {
        atomicAdd(&y[row], s);
        __threadfence();
        if (atomicAdd(&cnt[row], 1u) == (uint32_t)(nch - 1)) cnt[row] = 0;
    }
};

// z(row) = inv_b(row) * s (split rows zero beforehand); counts |row| into n_p
// for every row whose residue is positive.
struct EpiScaleCount {
    float *z;
    const float *inv_b;
    const int64_t *off;
    unsigned long long np = 0;
    __device__ void full(int64_t row, float s) {
        const float v = inv_b[row] * s;
        z[row] = v;
        if (v > 0.0f) np += (unsigned long long)(off[row + 1] - off[row]);
    }
    __device__ void partial(int64_t row, float s, int nch, uint32_t *cnt) {
        atomicAdd(&z[row], inv_b[row] * s);
        __threadfence();
        if (atomicAdd(&cnt[row], 1u) == (uint32_t)(nch - 1)) {
            cnt[row] = 0;
            if (atomicAdd(&z[row], 0.0f) > 0.0f) np += (unsigned long long)(off[row + 1] - off[row]);
        }
    }
};

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
    ctl->max_bits = 0;
    ctl->blocks_done = 0;
    ctl->n_p = 0;
    ctl->last_max = 1.0f;
}

// U side of a round (see file comment).  Also zeroes the split rows of z
// that the back kernel accumulates into.
__global__ void k_u_push(const Control *ctl, Control *ctl_w, float *__restrict__ r,
                         float *__restrict__ pi, float *__restrict__ rho, const float *__restrict__ c_d,
                         const float *__restrict__ c_s, const int64_t *__restrict__ off, int64_t n_u, float alpha,
                         float *__restrict__ z, const int32_t *__restrict__ zsplit, int64_t n_zsplit) {
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
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_zsplit; t += stride) z[zsplit[t]] = 0.0f;
    np = block_sum<unsigned long long>(np, lds);
    if (threadIdx.x == 0 && np) atomicAdd(&ctl_w->n_p, np);
}

// V and attribute rows: z = inv_b * (back CSR) rho.
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_back(const Control *ctl, Control *ctl_w, CsrView c,
                                                 const float *__restrict__ rho, float *z, const float *__restrict__ inv_b,
                                                 float *zero_arr, const int32_t *__restrict__ zero_rows,
                                                 int64_t n_zero) {
    __shared__ float prod[kWavesPerBlock][kItemEdges];
    __shared__ unsigned long long lds[4];
    if (ctl && ctl->done) return;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_zero; t += (int64_t)gridDim.x * blockDim.x)
        zero_arr[zero_rows[t]] = 0.0f;
    EpiScaleCount epi{z, inv_b, c.off};
    spmv_items<kUnit>(c, rho, prod[threadIdx.x >> 6], epi);
    if (ctl_w) {
        unsigned long long np = block_sum<unsigned long long>(epi.np, lds);
        if (threadIdx.x == 0 && np) atomicAdd(&ctl_w->n_p, np);
    }
}

// U rows: r += (fwd CSR) z, then the stop / switch rule in the last workgroup.
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_fwd(const Control *ctl, Control *ctl_w, CsrView c,
                                                const float *__restrict__ z, float *r, Rule rule) {
    __shared__ float prod[kWavesPerBlock][kItemEdges];
    __shared__ float ldsf[4];
    if (ctl->done) return;
    EpiAccumulate epi{r};
    spmv_items<kUnit>(c, z, prod[threadIdx.x >> 6], epi);
    const float m = block_max_f(epi.mx, ldsf);
    if (threadIdx.x == 0) {
        atomicMax(&ctl_w->max_bits, __float_as_uint(m));   // r >= 0, so bit order = value order
        __threadfence();
        if (atomicAdd(&ctl_w->blocks_done, 1u) == gridDim.x - 1) {
            __threadfence();
            const float mx = __uint_as_float(atomicAdd(&ctl_w->max_bits, 0u));
            const unsigned long long np = atomicAdd(&ctl_w->n_p, 0ull);
            const int iter = ctl_w->iter + 1;
            const float eps_f = ctl_w->eps_f;
            ctl_w->iter = iter;
            ctl_w->last_max = mx;
            ctl_w->max_bits = 0;
            ctl_w->blocks_done = 0;
            if (!(mx > eps_f)) {
                ctl_w->done = 1;
                ctl_w->status = 1;
            } else if (iter >= ctl_w->max_iters) {
                ctl_w->done = 1;
                ctl_w->status = 2;
            } else if (ctl_w->phase == 1) {
                // Budget of Algorithm 4 with the round count of Theorem 1's proof.
                const double t = (double)logf(mx / eps_f) * (double)rule.inv_log;
                if ((double)np >= rule.budget_scale * (t > 0.0 ? t : 0.0)) {
                    ctl_w->phase = 2;
                    ctl_w->theta = 0.0f;
                    ctl_w->switch_iter = iter;
                }
            }
        }
    }
}

// U rows, overwrite: y = (fwd CSR) z (split rows zero beforehand).
template <bool kUnit>
__global__ void __launch_bounds__(kBlock) k_fwd_overwrite(CsrView c, const float *__restrict__ z, float *y) {
    __shared__ float prod[kWavesPerBlock][kItemEdges];
    EpiOverwrite epi{y};
    spmv_items<kUnit>(c, z, prod[threadIdx.x >> 6], epi);
}

// Theorem 3 sweep, U side: acc += alpha y; rho = (c_d y, c_s y).
__global__ void k_lambda_u(const float *__restrict__ y, float *__restrict__ acc, float *__restrict__ rho,
                           const float *__restrict__ c_d, const float *__restrict__ c_s, int64_t n_u, float alpha,
                           float *__restrict__ z, const int32_t *__restrict__ zsplit, int64_t n_zsplit) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_u; j += stride) {
        const float x = y[j];
        acc[j] += alpha * x;
        rho[j] = c_d[j] * x;
        rho[n_u + j] = c_s[j] * x;
    }
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_zsplit; t += stride) z[zsplit[t]] = 0.0f;
}

__global__ void k_max_f32(const float *__restrict__ x, int64_t n, unsigned *out_bits) {
    __shared__ float ldsf[4];
    float m = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, x[i]);
    m = block_max_f(m, ldsf);
    if (threadIdx.x == 0) atomicMax(out_bits, __float_as_uint(m));
}

__global__ void k_sum_f64(const float *__restrict__ x, int64_t n, double *out) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += (double)x[i];
    s = block_sum<double>(s, lds);
    if (threadIdx.x == 0) atomicAdd(out, s);
}

unsigned elem_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (unsigned)g;
}

unsigned item_grid(int64_t n_items) {
    int64_t g = (n_items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (g < 1) g = 1;
    if (g > (int64_t)1 << 20) g = (int64_t)1 << 20;
    return (unsigned)g;
}

Rule make_rule(const Graph &g) {
    Rule r;
    r.alpha = (float)g.alpha;
    r.inv_log = (float)(1.0 / std::log(1.0 / (1.0 - g.alpha)));
    r.budget_scale = 2.0 * (double)(g.m_e + g.m_a);
    return r;
}

}  // namespace

void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f32, dim3(elem_grid(n)), dim3(kBlock), 0, s, p, v, n);
}

void single_query_init(Graph &g, int32_t source, float eps_f, int32_t max_iters, hipStream_t s) {
    launch_fill_f32(g.q_r, 0.0f, g.n_u, s);
    launch_fill_f32(g.q_pi, 0.0f, g.n_u, s);
    hipLaunchKernelGGL(k_query_init, dim3(1), dim3(64), 0, s, g.q_ctl, g.q_r, source, eps_f, max_iters);
    check_hip(hipGetLastError(), "query init");
}

void single_query_round(Graph &g, hipStream_t s) {
    hipLaunchKernelGGL(k_u_push, dim3(elem_grid(g.n_u)), dim3(kBlock), 0, s, g.q_ctl, g.q_ctl, g.q_r, g.q_pi, g.q_rho,
                       g.c_d, g.c_s, g.fwd.off, g.n_u, (float)g.alpha, g.q_z, g.back.split_rows, g.back.n_split);
    if (g.back.n_items > 0) {
        if (g.unit)
            hipLaunchKernelGGL(k_back<true>, dim3(item_grid(g.back.n_items)), dim3(kBlock), 0, s, g.q_ctl, g.q_ctl,
                               view(g.back), g.q_rho, g.q_z, g.inv_b, (float *)nullptr, (const int32_t *)nullptr,
                               (int64_t)0);
        else
            hipLaunchKernelGGL(k_back<false>, dim3(item_grid(g.back.n_items)), dim3(kBlock), 0, s, g.q_ctl, g.q_ctl,
                               view(g.back), g.q_rho, g.q_z, g.inv_b, (float *)nullptr, (const int32_t *)nullptr,
                               (int64_t)0);
    }
    const Rule rule = make_rule(g);
    if (g.unit)
        hipLaunchKernelGGL(k_fwd<true>, dim3(item_grid(g.fwd.n_items)), dim3(kBlock), 0, s, g.q_ctl, g.q_ctl,
                           view(g.fwd), g.q_z, g.q_r, rule);
    else
        hipLaunchKernelGGL(k_fwd<false>, dim3(item_grid(g.fwd.n_items)), dim3(kBlock), 0, s, g.q_ctl, g.q_ctl,
                           view(g.fwd), g.q_z, g.q_r, rule);
    check_hip(hipGetLastError(), "round launch");
}

void single_query_stats(Graph &g, double *sum_r, hipStream_t s) {
    double *d = nullptr;
    check_hip(hipMallocAsync((void **)&d, sizeof(double), s), "stats scratch");
    check_hip(hipMemsetAsync(d, 0, sizeof(double), s), "stats scratch");
    hipLaunchKernelGGL(k_sum_f64, dim3(elem_grid(g.n_u)), dim3(kBlock), 0, s, g.q_r, g.n_u, d);
    check_hip(hipMemcpyAsync(sum_r, d, sizeof(double), hipMemcpyDeviceToHost, s), "stats D2H");
    check_hip(hipFreeAsync(d, s), "stats scratch");
    check_hip(hipStreamSynchronize(s), "stats");
}

// Theorem 3 (Eq. 6): PI from the all-ones row vector for T rounds,
// lambda = max_i pi_T(u_i) + |U| (1-alpha)^T.
double compute_lambda(Graph &g, int T, hipStream_t s) {
    float *y = g.q_r, *acc = g.q_pi, *rho = g.q_rho, *z = g.q_z;
    launch_fill_f32(y, 1.0f, g.n_u, s);
    launch_fill_f32(acc, 0.0f, g.n_u, s);
    for (int t = 0; t < T; ++t) {
        hipLaunchKernelGGL(k_lambda_u, dim3(elem_grid(g.n_u)), dim3(kBlock), 0, s, y, acc, rho, g.c_d, g.c_s, g.n_u,
                           (float)g.alpha, z, g.back.split_rows, g.back.n_split);
        if (g.back.n_items > 0) {
            if (g.unit)
                hipLaunchKernelGGL(k_back<true>, dim3(item_grid(g.back.n_items)), dim3(kBlock), 0, s,
                                   (const Control *)nullptr, (Control *)nullptr, view(g.back), rho, z, g.inv_b, y,
                                   g.fwd.split_rows, g.fwd.n_split);
            else
                hipLaunchKernelGGL(k_back<false>, dim3(item_grid(g.back.n_items)), dim3(kBlock), 0, s,
                                   (const Control *)nullptr, (Control *)nullptr, view(g.back), rho, z, g.inv_b, y,
                                   g.fwd.split_rows, g.fwd.n_split);
        } else {
            launch_fill_f32(y, 0.0f, g.n_u, s);
        }
        if (g.unit)
            hipLaunchKernelGGL(k_fwd_overwrite<true>, dim3(item_grid(g.fwd.n_items)), dim3(kBlock), 0, s, view(g.fwd),
                               z, y);
        else
            hipLaunchKernelGGL(k_fwd_overwrite<false>, dim3(item_grid(g.fwd.n_items)), dim3(kBlock), 0, s,
                               view(g.fwd), z, y);
        check_hip(hipGetLastError(), "lambda launch");
    }
    unsigned *d = nullptr;
    check_hip(hipMalloc(&d, sizeof(unsigned)), "lambda scratch");
    check_hip(hipMemsetAsync(d, 0, sizeof(unsigned), s), "lambda scratch");
    hipLaunchKernelGGL(k_max_f32, dim3(elem_grid(g.n_u)), dim3(kBlock), 0, s, acc, g.n_u, d);
    unsigned bits = 0;
    check_hip(hipMemcpyAsync(&bits, d, sizeof(unsigned), hipMemcpyDeviceToHost, s), "lambda D2H");
    check_hip(hipStreamSynchronize(s), "lambda");
    dfree(d);
    float mx;
    std::memcpy(&mx, &bits, sizeof(float));
    return (double)mx + (double)g.n_u * std::pow(1.0 - g.alpha, (double)T);
}

}  // namespace ahpp
