// Monte Carlo estimate of one AHPP row (Section 3.1, Lemma 1): pi(u, x) is
// the probability that an alpha-hidden walk from u stops at x.  A walk stops
// at its current node with probability alpha; otherwise it takes one step of
// P = (1 - beta) P_S + beta P_A: with probability 1 - beta a structural
// two-hop step u -> v -> u' (v drawn with weight w(u, v) among N(u), then u'
// with weight w(v, u') among N(v)), else an attribute two-hop step
// u -> a -> u' (a with weight w(u, a) among A(u), u' with weight w(u', a)
// among the holders of a).  A step from a node whose chosen part is empty
// ends the walk without a stop (those rows of Eq. 1 / Eq. 2 are zero, so the
// probability mass is lost there too).
//
// One walk per thread, counter-based randomness (SplitMix64, Steele, Lea and
// Flood 2014, one sequential stream per walk from a key and the walk id),
// weighted draws by binary search in per-row prefix sums (double: rows of
// millions of entries keep every weight distinguishable), and integer
// atomic counts of the stops: the counts depend only on the seed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

constexpr uint64_t kGoldenMc = 0x9E3779B97F4A7C15ull;

struct Walker {
    uint64_t s;
    __device__ double next() {
        s += kGoldenMc;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }
};

// First entry of [e0, e1) whose prefix sum exceeds t (the last one if none).
__device__ __forceinline__ int64_t draw(const double *__restrict__ cum, int64_t e0, int64_t e1, double t) {
    int64_t lo = e0, hi = e1 - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (cum[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct McArgs {
    const int64_t *__restrict__ f_off;     // fwd CSR (rows U)
    const int32_t *__restrict__ f_col;
    const int64_t *__restrict__ f_split;   // first attribute entry of each U row
    const double *__restrict__ f_cum;      // prefix sums of raw weights, restarting at the V/attribute split
    const int64_t *__restrict__ b_off;     // back CSR (rows V, then n_v + a)
    const int32_t *__restrict__ b_col;
    const double *__restrict__ b_cum;      // prefix sums of raw weights per row
    int64_t n_v;
    int32_t source;
    int64_t n_walks;
    uint64_t key;
    double alpha, beta;
    int max_steps;
    unsigned *count;                       // [n_u] stops per node
    unsigned long long *tally;             // [0] lost, [1] truncated, [2] steps
};

__global__ void __launch_bounds__(kBlock) k_walks(McArgs a) {
    unsigned long long lost = 0, trunc = 0, steps = 0;
    unsigned at_source = 0;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < a.n_walks;
         w += (int64_t)gridDim.x * blockDim.x) {
        Walker rng{a.key + (uint64_t)w * 0x100000000ull};
        int32_t u = a.source;
        int st = 0;
        for (;; ++st) {
            if (st == a.max_steps) {
                ++trunc;
                break;
            }
            if (rng.next() < a.alpha) {
                if (u == a.source) ++at_source;
                else atomicAdd(&a.count[u], 1u);
                break;
            }
            const bool attr = rng.next() >= 1.0 - a.beta;
            const int64_t r0 = a.f_off[u], r1 = a.f_off[u + 1], sp = a.f_split[u];
            const int64_t e0 = attr ? sp : r0, e1 = attr ? r1 : sp;
            if (e0 == e1) {  // no edge (or no attribute) to step along
                ++lost;
                break;
            }
            const int64_t e = draw(a.f_cum, e0, e1, rng.next() * a.f_cum[e1 - 1]);
            const int64_t x = a.f_col[e];  // V id, or n_v + attribute: the back row to step from
            const int64_t g0 = a.b_off[x], g1 = a.b_off[x + 1];
            const int64_t f = draw(a.b_cum, g0, g1, rng.next() * a.b_cum[g1 - 1]);
            u = a.b_col[f];
        }
        steps += (unsigned long long)st;
    }
    // The source is the most frequent stop: one atomic per wave for it.
    const unsigned long long src = wave_sum_u64((unsigned long long)at_source);
    const unsigned long long l = wave_sum_u64(lost), tr = wave_sum_u64(trunc), sp = wave_sum_u64(steps);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (src) atomicAdd(&a.count[a.source], (unsigned)src);
        if (l) atomicAdd(&a.tally[0], l);
        if (tr) atomicAdd(&a.tally[1], tr);
        if (sp) atomicAdd(&a.tally[2], sp);
    }
}

// Prefix sums of raw weights for one wave per row: U rows restart at the
// first attribute entry (found by the column, V ids come first in a row);
// back rows use w(u, x) = w'(u, x) / c(u) with c the coefficient folded in
// at load, recovered from the U row sums.
__global__ void k_fwd_prefix(const int64_t *off, const int32_t *col, const float *w, int64_t n_u, int64_t n_v,
                             int64_t *split, double *cum, double *d_u, double *s_u) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = wave0; u < n_u; u += n_waves) {
        const int64_t e0 = off[u], e1 = off[u + 1];
        if (lane == 0) {
            int64_t lo = e0, hi = e1;  // first entry with col >= n_v
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (col[mid] >= n_v) hi = mid; else lo = mid + 1;
            }
            split[u] = lo;
            double run = 0.0, dv = 0.0;
            for (int64_t e = e0; e < e1; ++e) {
                if (e == lo) {
                    dv = run;
                    run = 0.0;
                }
                run += w ? (double)w[e] : 1.0;
                cum[e] = run;
            }
            if (lo == e1) {
                dv = run;
                run = 0.0;
            }
            d_u[u] = dv;
            s_u[u] = run;
        }
    }
}

__global__ void k_back_prefix(const int64_t *off, const int32_t *col, const float *w, int64_t n_v, int64_t n_rows,
                              const double *d_u, const double *s_u, double alpha, double beta, double *cum) {
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    if ((threadIdx.x & 63) != 0) return;
    for (int64_t x = wave0; x < n_rows; x += n_waves) {
        double run = 0.0;
        const bool v_row = x < n_v;
        for (int64_t e = off[x]; e < off[x + 1]; ++e) {
            const int32_t u = col[e];
            const double c = v_row ? (1.0 - beta) * (1.0 - alpha) / d_u[u] : beta * (1.0 - alpha) / s_u[u];
            run += (double)w[e] / c;
            cum[e] = run;
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_zero_u32(unsigned *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Scores in input order: out[i] = count[u_new[i]] / walks.
__global__ void k_scores(const unsigned *count, const int32_t *u_new, int64_t n, double inv_walks, float *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)((double)count[u_new[i]] * inv_walks);
}

unsigned grid_waves(int64_t rows) {
    const int64_t g = (rows * 64 + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

void free_mc_tables(McTables &t) {
    for (void *p : {(void *)t.f_split, (void *)t.f_cum, (void *)t.b_cum}) dfree(p);
    t = McTables{};
}

void ensure_mc_tables(Graph &g, hipStream_t s) {
    McTables &t = g.mc;
    if (t.f_cum) return;
    try {
        t.f_split = (int64_t *)dev_alloc(g, (size_t)std::max<int64_t>(g.n_u, 1) * 8, "walk tables");
        t.f_cum = (double *)dev_alloc(g, (size_t)std::max<int64_t>(g.fwd.nnz, 1) * 8, "walk tables");
        t.b_cum = (double *)dev_alloc(g, (size_t)std::max<int64_t>(g.back.nnz, 1) * 8, "walk tables");
        double *d_u = nullptr, *s_u = nullptr;
        check_hip(hipMalloc(&d_u, (size_t)std::max<int64_t>(g.n_u, 1) * 8), "walk tables");
        check_hip(hipMalloc(&s_u, (size_t)std::max<int64_t>(g.n_u, 1) * 8), "walk tables");
        hipLaunchKernelGGL(k_fwd_prefix, dim3(grid_waves(g.n_u)), dim3(kBlock), 0, s, g.fwd.off, g.fwd.col, g.fwd.w,
                           g.n_u, g.n_v, t.f_split, t.f_cum, d_u, s_u);
        if (g.n_v + g.n_a > 0)
            hipLaunchKernelGGL(k_back_prefix, dim3(grid_waves(g.n_v + g.n_a)), dim3(kBlock), 0, s, g.back.off,
                               g.back.col, g.back.w, g.n_v, g.n_v + g.n_a, d_u, s_u, g.alpha, g.beta, t.b_cum);
        check_hip(hipGetLastError(), "walk tables");
        check_hip(hipStreamSynchronize(s), "walk tables");
        dfree(d_u);
        dfree(s_u);
    } catch (...) {
        free_mc_tables(t);
        throw;
    }
}

void mc_scores(const unsigned *count, const int32_t *u_new, int64_t n, int64_t n_walks, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scores, dim3(1024), dim3(kBlock), 0, s, count, u_new, n, 1.0 / (double)n_walks, out);
    check_hip(hipGetLastError(), "walk scores");
}

McResult mc_walks(Graph &g, int32_t source, int64_t n_walks, uint64_t seed, int max_steps, unsigned *count,
                  hipStream_t s) {
    ensure_mc_tables(g, s);
    unsigned long long *tally = nullptr;
    check_hip(hipMallocAsync((void **)&tally, 3 * 8, s), "walk tally");
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, tally, (int64_t)3);
    hipLaunchKernelGGL(k_zero_u32, dim3(1024), dim3(kBlock), 0, s, count, g.n_u);
    McArgs a{g.fwd.off, g.fwd.col, g.mc.f_split, g.mc.f_cum, g.back.off, g.back.col, g.mc.b_cum, g.n_v, source,
             n_walks, seed * 0xD1B54A32D192ED03ull + 0x2545F4914F6CDD1Dull, g.alpha, g.beta, max_steps, count, tally};
    const int64_t blocks = std::min<int64_t>((n_walks + kBlock - 1) / kBlock, (int64_t)g.n_cu * 64);
    hipLaunchKernelGGL(k_walks, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0, s, a);
    check_hip(hipGetLastError(), "walks launch");
    unsigned long long h[3];
    check_hip(hipMemcpyAsync(h, tally, sizeof(h), hipMemcpyDeviceToHost, s), "walk tally");
    check_hip(hipFreeAsync(tally, s), "walk tally");
    check_hip(hipStreamSynchronize(s), "walks");
    return McResult{(int64_t)h[0], (int64_t)h[1], (int64_t)h[2]};
}

}  // namespace ahpp
