// Device top-k of AHPP scores: the k nodes with the largest pi_hat > 0, the
// source excluded, ordered by score descending then id ascending (the top-k
// lists Section 5 builds from the scores).
//
// Every candidate node i gets the 64-bit key (bits(pi_hat(i)) << 32) | ~i.
// Scores are non-negative, so their IEEE bits order like their values, and ~i
// breaks ties toward the smaller id; all keys are distinct.  A most-significant
// -digit radix select (8 bits per pass, at most 8 passes, each a histogram over
// the scores) finds the k-th largest key; the keys at or above it are gathered
// and sorted by one workgroup with a bitonic network in LDS.  Queries of a
// batch run side by side (grid.y = query).
#include <hip/hip_runtime.h>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

struct SelectState {
    unsigned long long prefix;  // decided high bits of the k-th key
    int32_t shift;              // bit position of the digit of the next pass
    int32_t remaining;          // keys still to take at or below the prefix
    int32_t done;
    int32_t take_all;           // fewer than k candidates: take every one
    int32_t n_cand;
    int32_t pad;
    unsigned hist[256];
};

__device__ __forceinline__ bool candidate(const float *s, int64_t i, int32_t excl, unsigned long long *key) {
    const float v = s[i];
    if (!(v > 0.0f) || i == excl) return false;
    *key = ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(~(uint32_t)i);
    return true;
}

__global__ void k_sel_init(SelectState *st, int64_t n_q, int32_t k) {
    const int64_t q = blockIdx.x;
    if (q >= n_q) return;
    SelectState &S = st[q];
    S.hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        S.prefix = 0;
        S.shift = 56;
        S.remaining = k;
        S.done = 0;
        S.take_all = 0;
        S.n_cand = 0;
    }
}

__global__ void k_sel_hist(const float *scores, int64_t n, int64_t stride_q, const int32_t *excl_dev,
                           int32_t excl_one, SelectState *st) {
    __shared__ unsigned h[256];
    const int64_t q = blockIdx.y;
    SelectState &S = st[q];
    if (S.done) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const float *s = scores + q * stride_q;
    const int32_t excl = excl_dev ? excl_dev[q] : excl_one;
    const int shift = S.shift;
    const unsigned long long hi = shift >= 56 ? 0ull : (S.prefix >> (shift + 8));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key;
        if (!candidate(s, i, excl, &key)) continue;
        if (shift < 56 && (key >> (shift + 8)) != hi) continue;
        atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&S.hist[threadIdx.x], h[threadIdx.x]);
}

// One workgroup per query: choose the digit holding the k-th largest key.
__global__ void k_sel_pick(SelectState *st) {
    __shared__ unsigned lds[4];
    SelectState &S = st[blockIdx.x];
    if (S.done) return;
    // Thread t looks at digit d = 255 - t; `above` counts keys in digits > d.
    const int t = threadIdx.x, d = 255 - t;
    const int32_t rem = S.remaining;
    const int shift = S.shift;
    const unsigned mine = S.hist[d];
    unsigned tot;
    const unsigned above = block_exclusive_scan<unsigned>(mine, lds, &tot);
    S.hist[d] = 0;
    if (shift == 56 && (int64_t)tot <= rem) {
        if (t == 0) {
            S.take_all = 1;
            S.done = 1;
            S.remaining = (int32_t)tot;
        }
        return;
    }
    if ((int64_t)above < rem && (int64_t)above + mine >= rem) {  // exactly one thread
        const int32_t left = rem - (int32_t)above;
        S.prefix |= (unsigned long long)d << shift;
        S.remaining = left;
        if ((int32_t)mine == left || shift == 0) S.done = 1;
        else S.shift = shift - 8;
    }
}

__global__ void k_sel_collect(const float *scores, int64_t n, int64_t stride_q, const int32_t *excl_dev,
                              int32_t excl_one, SelectState *st, unsigned long long *cand, int32_t k) {
    const int64_t q = blockIdx.y;
    SelectState &S = st[q];
    const float *s = scores + q * stride_q;
    const int32_t excl = excl_dev ? excl_dev[q] : excl_one;
    const unsigned long long thr = S.take_all ? 0ull : S.prefix;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key;
        if (!candidate(s, i, excl, &key) || key < thr) continue;
        const int pos = atomicAdd(&S.n_cand, 1);
        if (pos < k) cand[q * (int64_t)k + pos] = key;
    }
}

// Bitonic sort (descending) of each query's candidates in LDS.
__global__ void k_sel_sort(SelectState *st, const unsigned long long *cand, int32_t k, int32_t *idx_out,
                           float *val_out, int32_t *n_out) {
    __shared__ unsigned long long a[kMaxTopK];
    const int64_t q = blockIdx.x;
    const int32_t nc = min(st[q].n_cand, k);
    int n2 = 1;
    while (n2 < nc) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) a[i] = i < nc ? cand[q * (int64_t)k + i] : 0ull;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const unsigned long long x = a[i], y = a[j];
                    if (desc ? (x < y) : (x > y)) {
                        a[i] = y;
                        a[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const unsigned long long key = a[i];
        idx_out[q * (int64_t)k + i] = (int32_t)(~(uint32_t)(key & 0xffffffffull));
        val_out[q * (int64_t)k + i] = __uint_as_float((uint32_t)(key >> 32));
    }
    if (threadIdx.x == 0) n_out[q] = nc;
}

}  // namespace

size_t topk_scratch_bytes(int64_t n_q) { return (size_t)n_q * (sizeof(SelectState) + kMaxTopK * 8) + 256; }

void topk_launch(const float *scores, int64_t n, int64_t stride_q, int64_t n_q, const int32_t *exclude_dev,
                 int32_t exclude_one, int32_t k, int32_t *idx_out, float *val_out, int32_t *n_out, void *scratch,
                 hipStream_t s) {
    SelectState *st = (SelectState *)scratch;
    unsigned long long *cand = (unsigned long long *)((char *)scratch + (size_t)n_q * sizeof(SelectState));
    int64_t gx = (n + kBlock * 8 - 1) / (kBlock * 8);
    if (gx < 1) gx = 1;
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_sel_init, dim3((unsigned)n_q), dim3(256), 0, s, st, n_q, k);
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)gx, (unsigned)n_q), dim3(256), 0, s, scores, n, stride_q,
                           exclude_dev, exclude_one, st);
        hipLaunchKernelGGL(k_sel_pick, dim3((unsigned)n_q), dim3(256), 0, s, st);
    }
    hipLaunchKernelGGL(k_sel_collect, dim3((unsigned)gx, (unsigned)n_q), dim3(256), 0, s, scores, n, stride_q,
                       exclude_dev, exclude_one, st, cand, k);
    hipLaunchKernelGGL(k_sel_sort, dim3((unsigned)n_q), dim3(256), 0, s, st, cand, k, idx_out, val_out, n_out);
    check_hip(hipGetLastError(), "top-k launch");
}

}  // namespace ahpp
