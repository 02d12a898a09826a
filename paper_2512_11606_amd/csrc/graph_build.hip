// Device-side construction of the AHPP graph store (once per graph).
//
// From the COO lists E and E_A (Section 2.1) this builds, in HBM:
//   fwd : CSR over U.  Row u holds its V neighbours N(u) (column v) followed by
//         its attributes A(u) (column n_v + a), each with its raw weight.
//   back: CSR over V then attributes.  Row v holds N(v) (column u); row
//         n_v + a holds A^-1(a) (column n_u + u, so that one gathered vector
//         of length 2 n_u serves both halves).
// and the per-node coefficients of the push (Eq. 1 and Eq. 2 denominators):
//   c_d[u]   = (1-beta)(1-alpha) / d(u),     c_s[u] = beta (1-alpha) / s(u),
//   inv_b[v] = 1 / d(v),                     inv_b[n_v + a] = 1 / t(a).
// Rows keep the input order of their entries: a stable LSD radix sort
// (4-bit digits) groups entries by row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <utility>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

constexpr int kSortItems = 8;                       // keys per thread
constexpr int kSortTile = kBlock * kSortItems;      // keys per workgroup
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

// ---------------------------------------------------------------- validation

// flags bit 0: edge id out of range, bit 1: edge weight <= 0 or not finite,
//       bit 2: attribute id out of range, bit 3: attribute value <= 0 or not
//       finite, bit 4: some weight differs from 1.
__global__ void k_validate(const int32_t *a, const int32_t *b, const float *w, int64_t m, int64_t na, int64_t nb,
                           int id_bit, int w_bit, unsigned *flags) {
    unsigned f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = a[i], y = b[i];
        if (x < 0 || x >= na || y < 0 || y >= nb) f |= 1u << id_bit;
        if (w) {
            float v = w[i];
            if (!(v > 0.0f) || !isfinite(v)) f |= 1u << w_bit;
            if (v != 1.0f) f |= 1u << 4;
        }
    }
    if (f) atomicOr(flags, f);
}

// Keys, columns and weights of the entries to sort.
__global__ void k_make_entries(const int32_t *row_ids, const int32_t *col_ids, const float *w, int64_t m,
                               int32_t col_offset, uint32_t key_offset, uint32_t *key, int32_t *col, float *wo) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = (uint32_t)row_ids[i] + key_offset;
        col[i] = col_ids[i] + col_offset;
        wo[i] = w ? w[i] : 1.0f;
    }
}

// ---------------------------------------------------------------- numbering

// cnt[ids[i]] += 1 (integer atomics: the counts do not depend on the order).
__global__ void k_count_ids(const int32_t *ids, int64_t m, unsigned *cnt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[ids[i]], 1u);
}

// The same for small id sets (n <= kLdsCountMax): each workgroup counts its
// share in LDS, then adds its nonzero counts to cnt (few global atomics per
// id even when a few ids take most entries).
constexpr int64_t kLdsCountMax = 12288;
__global__ void k_count_ids_lds(const int32_t *ids, int64_t m, int64_t n, unsigned *cnt) {
    extern __shared__ unsigned h[];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[ids[i]], 1u);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        if (h[i]) atomicAdd(&cnt[i], h[i]);
}

// Sort keys of ids 0..n-1: larger counts first; the stable sort keeps id
// order among equal counts.
__global__ void k_rank_keys(const unsigned *cnt, int64_t n, uint32_t *key, int32_t *id) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = ~cnt[i];
        id[i] = (int32_t)i;
    }
}

// new_of[order[j]] = j.
__global__ void k_invert(const int32_t *order, int64_t n, int32_t *new_of) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        new_of[order[j]] = (int32_t)j;
}

// ids[i] = new_of[ids[i]].
__global__ void k_remap(int32_t *ids, int64_t m, const int32_t *new_of) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        ids[i] = new_of[ids[i]];
}

// Zero-count entries: how many of the n counts are nonzero.
__global__ void k_count_nonzero(const unsigned *cnt, int64_t n, unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += cnt[i] != 0u;
    if (c) atomicAdd(out, c);
}

// ---------------------------------------------------------------- scan

__global__ void k_scan_partials(const unsigned long long *in, int64_t n, unsigned long long *part) {
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) s += in[base + j];
    s = block_sum<unsigned long long>(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Exclusive scan of `part` (n_part entries) by one workgroup, in place.
__global__ void k_scan_single(unsigned long long *part, int64_t n_part) {
    __shared__ unsigned long long lds[4];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < n_part; base += kBlock) {
        int64_t i = base + threadIdx.x;
        unsigned long long v = i < n_part ? part[i] : 0ull;
        unsigned long long tot;
        unsigned long long ex = block_exclusive_scan<unsigned long long>(v, lds, &tot);
        if (i < n_part) part[i] = carry + ex;
        carry += tot;
    }
}

__global__ void k_scan_apply(const unsigned long long *in, int64_t n, const unsigned long long *part,
                             unsigned long long *out) {
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    unsigned long long v[kScanItems];
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + j < n ? in[base + j] : 0ull;
        s += v[j];
    }
    unsigned long long tot;
    unsigned long long ex = block_exclusive_scan<unsigned long long>(s, lds, &tot) + part[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
}

// Exclusive scan of n unsigned 64-bit values (in may equal out).
void exclusive_scan_u64(const unsigned long long *in, unsigned long long *out, int64_t n,
                        unsigned long long *part, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kBlock), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part, out);
    check_hip(hipGetLastError(), "scan launch");
}

// ---------------------------------------------------------------- radix sort

// Digit histogram of every tile, stored digit-major: cnt[d * n_tiles + t].
__global__ void k_radix_count(const uint32_t *key, int64_t n, int shift, unsigned long long *cnt, int64_t n_tiles) {
    __shared__ unsigned h[16];
    if (threadIdx.x < 16) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
        if (base + j < n) atomicAdd(&h[(key[base + j] >> shift) & 15u], 1u);
    __syncthreads();
    if (threadIdx.x < 16) cnt[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: thread t owns keys [t*8, t*8+8) of the tile, so
// (thread, item) order is input order; within a digit, keys keep that order.
__global__ void k_radix_scatter(const uint32_t *key, const int32_t *col, const float *w, int64_t n, int shift,
                                const unsigned long long *dig_off, int64_t n_tiles, uint32_t *key_o, int32_t *col_o,
                                float *w_o) {
    __shared__ unsigned cnt[16 * kBlock];  // [digit][thread]
    __shared__ unsigned dstart[16];
    __shared__ unsigned lds[4];
    const int tid = threadIdx.x;
    for (int d = 0; d < 16; ++d) cnt[d * kBlock + tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)tid * kSortItems;
    uint32_t k[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        k[j] = base + j < n ? key[base + j] : 0xffffffffu;
        if (base + j < n) cnt[((k[j] >> shift) & 15u) * kBlock + tid] += 1;
    }
    __syncthreads();
    // Exclusive scan over cnt in digit-major order: thread tid scans entries
    // [tid*16, tid*16+16).
    unsigned v[16];
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        v[j] = cnt[tid * 16 + j];
        s += v[j];
    }
    unsigned tot;
    unsigned ex = block_exclusive_scan<unsigned>(s, lds, &tot);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        cnt[tid * 16 + j] = ex;
        ex += v[j];
    }
    __syncthreads();
    // Tile-local start of digit d, read before any thread advances its slots.
    if (tid < 16) dstart[tid] = cnt[tid * kBlock];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (base + j >= n) continue;
        unsigned d = (k[j] >> shift) & 15u;
        unsigned local = cnt[d * kBlock + tid] - dstart[d];
        cnt[d * kBlock + tid] += 1;
        int64_t pos = (int64_t)dig_off[(int64_t)d * n_tiles + blockIdx.x] + local;
        key_o[pos] = k[j];
        col_o[pos] = col[base + j];
        if (w) w_o[pos] = w[base + j];
    }
}

// off[r] = first position whose key is >= r, for r in [0, n_rows]; key sorted.
__global__ void k_offsets(const uint32_t *key, int64_t n, int64_t n_rows, int64_t *off) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t prev = i == 0 ? -1 : (int64_t)key[i - 1];
        int64_t cur = i == n ? n_rows : (int64_t)key[i];
        for (int64_t r = prev + 1; r <= cur; ++r) off[r] = i;
    }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Row sums of fwd in double precision, one wave per row: d(u) over columns
// < n_v (Eq. 1 denominator), s(u) over the attribute columns (Eq. 2);
// stores c_d = (1-beta)(1-alpha)/d(u) and c_s = beta(1-alpha)/s(u).
__global__ void k_fwd_coeffs(const int64_t *off, const int32_t *col, const float *w, int64_t n_u, int64_t n_v,
                             double alpha, double beta, double *c_d, double *c_s, unsigned long long *dangling) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long dang = 0;
    for (int64_t u = wave0; u < n_u; u += n_waves) {
        double d = 0.0, s = 0.0;
        for (int64_t p = off[u] + lane; p < off[u + 1]; p += 64) {
            double x = w ? (double)w[p] : 1.0;
            if (col[p] < n_v) d += x; else s += x;
        }
        d = wave_sum_f64(d);
        s = wave_sum_f64(s);
        if (lane == 0) {
            c_d[u] = d > 0 ? (1.0 - beta) * (1.0 - alpha) / d : 0.0;
            c_s[u] = s > 0 ? beta * (1.0 - alpha) / s : 0.0;
            if (!(d > 0) || !(s > 0)) dang += 1;
        }
    }
    if (dang) atomicAdd(dangling, dang);
}

// One wave per back row x: inv_b = 1/d(v) (V rows) or 1/t(a) (attribute rows)
// from the raw weights, then each weight becomes w(u,x) c_d(u) (V rows) or
// w(u,x) c_s(u) (attribute rows), rounded once from double.
__global__ void k_back_coeffs(const int64_t *off, const int32_t *col, float *w, int64_t n_v, int64_t n_rows,
                              const double *c_d, const double *c_s, float *inv_b) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave0; r < n_rows; r += n_waves) {
        double d = 0.0;
        for (int64_t p = off[r] + lane; p < off[r + 1]; p += 64) d += (double)w[p];
        d = wave_sum_f64(d);
        if (lane == 0) inv_b[r] = d > 0 ? (float)(1.0 / d) : 0.0f;
        const double *c = r < n_v ? c_d : c_s;
        for (int64_t p = off[r] + lane; p < off[r + 1]; p += 64) w[p] = (float)((double)w[p] * c[col[p]]);
    }
}

unsigned grid_for(int64_t n, int per_block = kBlock, unsigned cap = 65536u) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// Builds the wave schedule of a CSR from its host copy of the offsets; rows
// with skip[r] set get no item (a pack of short rows ends before them).
void build_items(const std::vector<int64_t> &off, std::vector<WorkItem> &items, std::vector<SplitRow> &split,
                 int32_t &max_len, const std::vector<uint8_t> *skip = nullptr) {
    const int64_t n_rows = (int64_t)off.size() - 1;
    items.clear();
    split.clear();
    max_len = 0;
    int64_t r = 0;
    while (r < n_rows) {
        int64_t len = off[r + 1] - off[r];
        max_len = (int32_t)std::max<int64_t>(max_len, len);
        if (skip && (*skip)[r]) {
            ++r;
            continue;
        }
        if (len > kShortRow) {
            int64_t chunks = (len + kItemEdges - 1) / kItemEdges;
            if (chunks > 1) split.push_back(SplitRow{(int32_t)r, (int32_t)items.size(), (int32_t)chunks, 0});
            for (int64_t c = 0; c < chunks; ++c) items.push_back(WorkItem{(int32_t)r, (int32_t)(-c)});
            ++r;
            continue;
        }
        // Pack consecutive short rows.
        int64_t r1 = r, e = 0;
        while (r1 < n_rows && r1 - r < kMaxRowsPerItem && !(skip && (*skip)[r1])) {
            int64_t l = off[r1 + 1] - off[r1];
            if (l > kShortRow || e + l > kItemEdges) break;
            e += l;
            ++r1;
        }
        items.push_back(WorkItem{(int32_t)r, (int32_t)(r1 - r)});
        r = r1;
    }
}

// Sorts (key, col, w) by key (stable) and builds offsets + schedule.
// Stable LSD radix sort (4-bit digits) of m (key, col[, w]) triples by key,
// keys below 2^key_bits; the sorted triples end in the same buffers.
void sort_by_key(uint32_t *key, int32_t *col, float *w, int64_t m, int key_bits, hipStream_t s) {
    if (m <= 0) return;
    const int64_t n_tiles = (m + kSortTile - 1) / kSortTile;
    const int64_t n_cnt = 16 * n_tiles;
    DevTemp<uint32_t> key2((size_t)m, "sort buffer");
    DevTemp<int32_t> col2((size_t)m, "sort buffer");
    DevTemp<float> w2(w ? (size_t)m : 0, "sort buffer");
    DevTemp<unsigned long long> cnt((size_t)n_cnt, "sort counts");
    DevTemp<unsigned long long> part((size_t)((n_cnt + kScanTile - 1) / kScanTile + 1), "scan partials");
    const int passes = (key_bits + 3) / 4;
    uint32_t *ki = key, *ko = key2.get();
    int32_t *ci = col, *co = col2.get();
    float *wi = w, *wo = w2.get();
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_radix_count, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, ki, m, 4 * p, cnt.get(),
                           n_tiles);
        exclusive_scan_u64(cnt.get(), cnt.get(), n_cnt, part.get(), s);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, ki, ci, wi, m, 4 * p,
                           cnt.get(), n_tiles, ko, co, wo);
        check_hip(hipGetLastError(), "radix sort launch");
        std::swap(ki, ko);
        std::swap(ci, co);
        std::swap(wi, wo);
    }
    if (ki != key) {
        check_hip(hipMemcpyAsync(key, ki, (size_t)m * 4, hipMemcpyDeviceToDevice, s), "sort copy");
        check_hip(hipMemcpyAsync(col, ci, (size_t)m * 4, hipMemcpyDeviceToDevice, s), "sort copy");
        if (w) check_hip(hipMemcpyAsync(w, wi, (size_t)m * 4, hipMemcpyDeviceToDevice, s), "sort copy");
    }
    check_hip(hipStreamSynchronize(s), "sort");
}

// CSR of m entries (row key, column, weight).  With n_cols > 0 the entries of
// every row are put in column order (a stable sort by column first), which
// under the device numbering puts a row's most referenced columns side by
// side for the lanes of one load; otherwise rows keep the input order.
void build_csr(Graph &g, DevCsr &c, int64_t n_rows, uint32_t *key, int32_t *col, float *w, int64_t m, bool keep_w,
               hipStream_t s, int64_t n_cols = 0, bool with_items = true) {
    c.n_rows = n_rows;
    c.nnz = m;
    c.off = (int64_t *)dev_alloc(g, (size_t)(n_rows + 1) * sizeof(int64_t), "csr offsets");
    // The padding lets a group of scalar loads run past the last row's end.
    c.col = (int32_t *)dev_alloc(g, (size_t)(m + kCsrPad) * sizeof(int32_t), "csr columns");
    check_hip(hipMemsetAsync(c.col + m, 0, kCsrPad * sizeof(int32_t), s), "csr padding");
    if (keep_w) {
        c.w = (float *)dev_alloc(g, (size_t)(m + kCsrPad) * sizeof(float), "csr weights");
        check_hip(hipMemsetAsync(c.w + m, 0, kCsrPad * sizeof(float), s), "csr padding");
    }
    if (m > 0) {
        // Columns are non-negative, so their bits order like unsigned keys.
        if (n_cols > 0)
            sort_by_key(reinterpret_cast<uint32_t *>(col), reinterpret_cast<int32_t *>(key), w, m, bits_for(n_cols), s);
        sort_by_key(key, col, w, m, bits_for(n_rows), s);
        hipLaunchKernelGGL(k_offsets, dim3(grid_for(m + 1)), dim3(kBlock), 0, s, key, m, n_rows, c.off);
        check_hip(hipMemcpyAsync(c.col, col, (size_t)m * 4, hipMemcpyDeviceToDevice, s), "csr copy");
        if (c.w) check_hip(hipMemcpyAsync(c.w, w, (size_t)m * 4, hipMemcpyDeviceToDevice, s), "csr copy");
        check_hip(hipStreamSynchronize(s), "csr build");
    } else {
        check_hip(hipMemsetAsync(c.off, 0, (size_t)(n_rows + 1) * sizeof(int64_t), s), "csr offsets");
    }
    if (!with_items) return;
    // Wave schedule (host side: a linear greedy pass over the offsets).
    std::vector<int64_t> off((size_t)n_rows + 1);
    check_hip(hipMemcpyAsync(off.data(), c.off, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s), "offsets D2H");
    check_hip(hipStreamSynchronize(s), "offsets D2H");
    std::vector<WorkItem> items;
    std::vector<SplitRow> split;
    build_items(off, items, split, c.max_row_len);
    if ((int64_t)items.size() > (int64_t)INT32_MAX) throw Failure{-1, "ahpp_graph_load: schedule exceeds int32 items"};
    c.n_items = (int64_t)items.size();
    c.n_split = (int64_t)split.size();
    std::vector<int64_t> ie0(items.size());
    std::vector<int32_t> ine(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        const WorkItem &it = items[i];
        if (it.n > 0) {
            ie0[i] = off[it.row];
            ine[i] = (int32_t)(off[it.row + it.n] - off[it.row]);
        } else {
            const int64_t rb = off[it.row], len = off[it.row + 1] - rb, first = (int64_t)(-it.n) * kItemEdges;
            ie0[i] = rb + first;
            const int32_t ne = (int32_t)std::min<int64_t>(len - first, kItemEdges);
            ine[i] = len <= kItemEdges ? ne : -ne;
        }
    }
    c.item_e0 = (int64_t *)dev_alloc(g, std::max<size_t>(items.size(), 1) * 8, "schedule");
    c.item_ne = (int32_t *)dev_alloc(g, std::max<size_t>(items.size(), 1) * 4, "schedule");
    if (!items.empty()) {
        check_hip(hipMemcpyAsync(c.item_e0, ie0.data(), ie0.size() * 8, hipMemcpyHostToDevice, s), "schedule H2D");
        check_hip(hipMemcpyAsync(c.item_ne, ine.data(), ine.size() * 4, hipMemcpyHostToDevice, s), "schedule H2D");
    }
    c.items = (WorkItem *)dev_alloc(g, std::max<size_t>(items.size(), 1) * sizeof(WorkItem), "schedule");
    c.split = (SplitRow *)dev_alloc(g, std::max<size_t>(split.size(), 1) * sizeof(SplitRow), "split rows");
    if (!items.empty())
        check_hip(hipMemcpyAsync(c.items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s),
                  "schedule H2D");
    if (!split.empty())
        check_hip(hipMemcpyAsync(c.split, split.data(), split.size() * sizeof(SplitRow), hipMemcpyHostToDevice, s),
                  "split H2D");
    check_hip(hipStreamSynchronize(s), "schedule upload");
}

// Numbers the ids 0..n-1 of one node set by descending reference count
// (the entries of `lists` that name them), ties by id: new_of[id] = its
// number.  Returns how many ids have a nonzero count (they come first).
int64_t number_by_count(Graph &g, int64_t n, std::initializer_list<std::pair<const int32_t *, int64_t>> lists,
                        int32_t *new_of, hipStream_t s) {
    if (n <= 0) return 0;
    DevTemp<unsigned> cnt_((size_t)n, "numbering");
    DevTemp<uint32_t> key_((size_t)n, "numbering");
    DevTemp<int32_t> order_((size_t)n, "numbering");
    DevTemp<unsigned long long> nz_(1, "numbering");
    unsigned *cnt = cnt_.get();
    uint32_t *key = key_.get();
    int32_t *order = order_.get();
    unsigned long long *nz = nz_.get();
    check_hip(hipMemsetAsync(cnt, 0, (size_t)n * 4, s), "numbering");
    check_hip(hipMemsetAsync(nz, 0, 8, s), "numbering");
    for (const auto &l : lists) {
        if (l.second <= 0) continue;
        if (n <= kLdsCountMax)
            hipLaunchKernelGGL(k_count_ids_lds, dim3(std::min<unsigned>(grid_for(l.second), 1024u)), dim3(kBlock),
                               (size_t)n * sizeof(unsigned), s, l.first, l.second, n, cnt);
        else
            hipLaunchKernelGGL(k_count_ids, dim3(grid_for(l.second)), dim3(kBlock), 0, s, l.first, l.second, cnt);
    }
    hipLaunchKernelGGL(k_count_nonzero, dim3(grid_for(n)), dim3(kBlock), 0, s, cnt, n, nz);
    hipLaunchKernelGGL(k_rank_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, cnt, n, key, order);
    check_hip(hipGetLastError(), "numbering launch");
    sort_by_key(key, order, nullptr, n, 32, s);
    hipLaunchKernelGGL(k_invert, dim3(grid_for(n)), dim3(kBlock), 0, s, order, n, new_of);
    check_hip(hipGetLastError(), "numbering launch");
    unsigned long long n_nz = 0;
    check_hip(hipMemcpyAsync(&n_nz, nz, 8, hipMemcpyDeviceToHost, s), "numbering");
    check_hip(hipStreamSynchronize(s), "numbering");
    (void)g;
    return (int64_t)n_nz;
}

// Picks the hot rows of the back CSR (the kHotMax longest rows with at least
// kHotMinLen entries, longest first; AHPP_HOT_ROWS=<n> lowers the cap, 0
// turns them off), builds their dense MFMA weights and the back schedule
// without them.  The dense block (6 bytes per hot row and U node, rounded up
// to whole chunks) is used when it takes at most a quarter of the device's
// memory, a fixed property of the device, so whether a graph has hot rows
// (and so the order of its sums) does not depend on what else is allocated.
void build_hot(Graph &g, hipStream_t s) {
    HotSet &h = g.hot;
    int cap = kHotMax;
    if (const char *e = std::getenv("AHPP_HOT_ROWS")) cap = std::max(0, std::min(kHotMax, std::atoi(e)));
    const int64_t n_rows = g.back.n_rows;
    if (cap == 0 || n_rows == 0 || g.back.nnz == 0) return;
    size_t free_b = 0, total_b = 0;
    check_hip(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if ((double)hot_dense_bytes(g) > 0.25 * (double)total_b) return;
    std::vector<int64_t> off((size_t)n_rows + 1);
    check_hip(hipMemcpyAsync(off.data(), g.back.off, off.size() * 8, hipMemcpyDeviceToHost, s), "hot rows");
    check_hip(hipStreamSynchronize(s), "hot rows");
    std::vector<int32_t> order;
    for (int64_t r = 0; r < n_rows; ++r)
        if (off[r + 1] - off[r] >= kHotMinLen) order.push_back((int32_t)r);
    if (order.empty()) return;
    // Longest first, ties by row id.
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
    if ((int)order.size() > cap) order.resize(cap);
    const int n = (int)order.size();
    std::vector<int32_t> len(n);
    std::vector<uint8_t> skip((size_t)n_rows, 0);
    int64_t m = 0;
    for (int i = 0; i < n; ++i) {
        len[i] = (int32_t)(off[order[i] + 1] - off[order[i]]);
        m += len[i];
        skip[order[i]] = 1;
    }
    h.n = n;
    h.rows = (int32_t *)dev_alloc(g, (size_t)n * 4, "hot rows");
    h.len = (int32_t *)dev_alloc(g, (size_t)n * 4, "hot rows");
    check_hip(hipMemcpyAsync(h.rows, order.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "hot rows");
    check_hip(hipMemcpyAsync(h.len, len.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "hot rows");
    build_hot_dense(g, s);
    // Back schedule without the hot rows.
    std::vector<WorkItem> items;
    std::vector<SplitRow> split;
    int32_t max_len = 0;
    build_items(off, items, split, max_len, &skip);
    h.n_cold_items = (int64_t)items.size();
    h.n_cold_split = (int64_t)split.size();
    h.cold_items = (WorkItem *)dev_alloc(g, std::max<size_t>(items.size(), 1) * sizeof(WorkItem), "cold schedule");
    h.cold_split = (SplitRow *)dev_alloc(g, std::max<size_t>(split.size(), 1) * sizeof(SplitRow), "cold schedule");
    if (!items.empty())
        check_hip(hipMemcpyAsync(h.cold_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s),
                  "cold schedule");
    if (!split.empty())
        check_hip(hipMemcpyAsync(h.cold_split, split.data(), split.size() * sizeof(SplitRow), hipMemcpyHostToDevice,
                                 s), "cold schedule");
    h.cold_nnz = g.back.nnz - m;
    h.cold_rows = n_rows - n;
    check_hip(hipStreamSynchronize(s), "hot rows");
}

}  // namespace

namespace {
// With AHPP_LOAD_TRACE=1 the load prints the time of each phase to stderr
// (the stream is synchronized at each mark).
struct LoadTrace {
    bool on;
    std::chrono::steady_clock::time_point t;
    LoadTrace() : on(std::getenv("AHPP_LOAD_TRACE") && std::atoi(std::getenv("AHPP_LOAD_TRACE")) == 1),
                  t(std::chrono::steady_clock::now()) {}
    void mark(const char *what, hipStream_t s) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[ahpp load] %-28s %9.1f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};
}  // namespace

void build_graph(Graph &g, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                 const int32_t *aa, const float *aw, const KeyInput &kin, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    LoadTrace trace;
    const int64_t m_e = g.m_e, m_a = g.m_a, m = m_e + m_a;
    {  // The COO upload and the entry scratch end with the block.
        // Upload COO (a missing weight array means every weight is 1).
        auto n_of = [](int64_t n, const void *src) { return (size_t)(src && n > 0 ? n : 0); };
        DevTemp<int32_t> eu_(n_of(m_e, eu), "edge upload"), ev_(n_of(m_e, ev), "edge upload");
        DevTemp<float> ew_(n_of(m_e, ew), "edge upload");
        DevTemp<int32_t> au_(n_of(m_a, au), "assoc upload"), aa_(n_of(m_a, aa), "assoc upload");
        DevTemp<float> aw_(n_of(m_a, aw), "assoc upload");
        int32_t *d_eu = eu_.get(), *d_ev = ev_.get(), *d_au = au_.get(), *d_aa = aa_.get();
        float *d_ew = ew_.get(), *d_aw = aw_.get();
        auto up = [&](void *dst, const void *src, size_t n, const char *what) {
            if (n) check_hip(hipMemcpyAsync(dst, src, n * 4, hipMemcpyHostToDevice, s), what);
        };
        up(d_eu, eu, n_of(m_e, eu), "edge upload");
        up(d_ev, ev, n_of(m_e, ev), "edge upload");
        up(d_ew, ew, n_of(m_e, ew), "edge upload");
        up(d_au, au, n_of(m_a, au), "assoc upload");
        up(d_aa, aa, n_of(m_a, aa), "assoc upload");
        up(d_aw, aw, n_of(m_a, aw), "assoc upload");
        DevTemp<unsigned> flags_(1, "flags");
        unsigned *d_flags = flags_.get();
        check_hip(hipMemsetAsync(d_flags, 0, sizeof(unsigned), s), "flags");
        if (m_e > 0)
            hipLaunchKernelGGL(k_validate, dim3(grid_for(m_e)), dim3(kBlock), 0, s, d_eu, d_ev, d_ew, m_e, g.n_u,
                               g.n_v, 0, 1, d_flags);
        if (m_a > 0)
            hipLaunchKernelGGL(k_validate, dim3(grid_for(m_a)), dim3(kBlock), 0, s, d_au, d_aa, d_aw, m_a, g.n_u,
                               g.n_a, 2, 3, d_flags);
        unsigned flags = 0;
        check_hip(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, s), "flags D2H");
        check_hip(hipStreamSynchronize(s), "validation");
        if (flags & 15u) {
            std::string msg = "ahpp_graph_load:";
            if (flags & 1u) msg += " edge id out of range;";
            if (flags & 2u) msg += " edge weight not positive and finite;";
            if (flags & 4u) msg += " attribute association id out of range;";
            if (flags & 8u) msg += " attribute value not positive and finite;";
            throw Failure{-1, msg};
        }
        g.unit = !(flags & 16u);
        trace.mark("upload + validation", s);
        coo_key_device(kin, d_eu, d_ev, d_ew, d_au, d_aa, d_aw, g.key, s);
        trace.mark("input key", s);

        // Device numbering of U, V and the attributes: by descending number of
        // CSR entries that name the node, ties by input id.  The random gathers
        // of a round then find the most referenced nodes packed together (more
        // of them per cache line).  A V node without an edge is never read and
        // never receives residue: it gets no row (it sorts last and is cut).
        // Only U numbers leave the library, and they are mapped back on the way
        // out (u_new, u_new_host).
        g.n_v_input = g.n_v;
        g.u_new = (int32_t *)dev_alloc(g, (size_t)g.n_u * 4, "U numbering");
        number_by_count(g, g.n_u, {{d_eu, m_e}, {d_au, m_a}}, g.u_new, s);
        DevTemp<int32_t> v_new_((size_t)std::max<int64_t>(g.n_v, 0), "V numbering");
        DevTemp<int32_t> a_new_((size_t)std::max<int64_t>(g.n_a, 0), "attribute numbering");
        int32_t *v_new = v_new_.get(), *a_new = a_new_.get();
        const int64_t v_rows = number_by_count(g, g.n_v, {{d_ev, m_e}}, v_new, s);
        number_by_count(g, g.n_a, {{d_aa, m_a}}, a_new, s);
        if (m_e > 0) {
            hipLaunchKernelGGL(k_remap, dim3(grid_for(m_e)), dim3(kBlock), 0, s, d_eu, m_e, g.u_new);
            hipLaunchKernelGGL(k_remap, dim3(grid_for(m_e)), dim3(kBlock), 0, s, d_ev, m_e, v_new);
        }
        if (m_a > 0) {
            hipLaunchKernelGGL(k_remap, dim3(grid_for(m_a)), dim3(kBlock), 0, s, d_au, m_a, g.u_new);
            hipLaunchKernelGGL(k_remap, dim3(grid_for(m_a)), dim3(kBlock), 0, s, d_aa, m_a, a_new);
        }
        check_hip(hipGetLastError(), "numbering launch");
        g.u_new_host.resize((size_t)g.n_u);
        check_hip(hipMemcpyAsync(g.u_new_host.data(), g.u_new, (size_t)g.n_u * 4, hipMemcpyDeviceToHost, s),
                  "numbering");
        check_hip(hipStreamSynchronize(s), "numbering");
        g.n_v = v_rows;
        trace.mark("numbering", s);

        // Entries of both CSRs.
        DevTemp<uint32_t> key_((size_t)m, "entries");
        DevTemp<int32_t> col_((size_t)m, "entries");
        DevTemp<float> w_((size_t)m, "entries");
        uint32_t *key = key_.get();
        int32_t *col = col_.get();
        float *w = w_.get();
        // fwd: rows U; edges (col v) then associations (col n_v + a).
        if (m_e > 0)
            hipLaunchKernelGGL(k_make_entries, dim3(grid_for(m_e)), dim3(kBlock), 0, s, d_eu, d_ev, d_ew, m_e, 0, 0u,
                               key, col, w);
        if (m_a > 0)
            hipLaunchKernelGGL(k_make_entries, dim3(grid_for(m_a)), dim3(kBlock), 0, s, d_au, d_aa, d_aw, m_a,
                               (int32_t)g.n_v, 0u, key + m_e, col + m_e, w + m_e);
        build_csr(g, g.fwd, g.n_u, key, col, w, m, !g.unit, s, g.n_v + g.n_a);
        trace.mark("U rows (sort + schedule)", s);
        // back: rows V then attributes (row n_v + a); columns are U ids.
        if (m_e > 0)
            hipLaunchKernelGGL(k_make_entries, dim3(grid_for(m_e)), dim3(kBlock), 0, s, d_ev, d_eu, d_ew, m_e, 0, 0u,
                               key, col, w);
        if (m_a > 0)
            hipLaunchKernelGGL(k_make_entries, dim3(grid_for(m_a)), dim3(kBlock), 0, s, d_aa, d_au, d_aw, m_a, 0,
                               (uint32_t)g.n_v, key + m_e, col + m_e, w + m_e);
        build_csr(g, g.back, g.n_v + g.n_a, key, col, w, m, true, s, g.n_u);
        trace.mark("V/attribute rows", s);
    }

    // Coefficients: 1/d(u), 1/s(u) in double, then inv_b and the back weights
    // w(u,x) * c(u) with c = (1-beta)(1-alpha)/d(u) or beta(1-alpha)/s(u).
    g.inv_b = (float *)dev_alloc(g, (size_t)std::max<int64_t>(g.n_v + g.n_a, 1) * 4, "inv_b");
    DevTemp<double> cd_((size_t)std::max<int64_t>(g.n_u, 1), "coefficients");
    DevTemp<double> cs_((size_t)std::max<int64_t>(g.n_u, 1), "coefficients");
    DevTemp<unsigned long long> dang_(1, "dangling");
    double *cd = cd_.get(), *cs = cs_.get();
    unsigned long long *d_dang = dang_.get();
    check_hip(hipMemsetAsync(d_dang, 0, 8, s), "dangling");
    hipLaunchKernelGGL(k_fwd_coeffs, dim3(grid_for(g.n_u * 64)), dim3(kBlock), 0, s, g.fwd.off, g.fwd.col, g.fwd.w,
                       g.n_u, g.n_v, g.alpha, g.beta, cd, cs, d_dang);
    if (g.n_v + g.n_a > 0)
        hipLaunchKernelGGL(k_back_coeffs, dim3(grid_for((g.n_v + g.n_a) * 64)), dim3(kBlock), 0, s, g.back.off,
                           g.back.col, g.back.w, g.n_v, g.n_v + g.n_a, cd, cs, g.inv_b);
    check_hip(hipGetLastError(), "coefficient launch");
    unsigned long long dang = 0;
    check_hip(hipMemcpyAsync(&dang, d_dang, 8, hipMemcpyDeviceToHost, s), "dangling D2H");
    check_hip(hipStreamSynchronize(s), "coefficients");
    g.dangling_u = (int64_t)dang;
    trace.mark("coefficients", s);
    build_hot(g, s);
    trace.mark("hot rows", s);
    g.load_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void free_csr(DevCsr &c) {
    dfree(c.off); dfree(c.col); dfree(c.w); dfree(c.items); dfree(c.split); dfree(c.item_e0); dfree(c.item_ne);
    c = DevCsr{};
}

void free_graph(Graph &g) {
    if (g.single_round_graph) (void)hipGraphExecDestroy(g.single_round_graph);
    g.single_round_graph = nullptr;
    if (g.cap_stream) (void)hipStreamDestroy(g.cap_stream);
    g.cap_stream = nullptr;
    free_csr(g.fwd);
    free_csr(g.back);
    free_mc_tables(g.mc);
    for (void *p : {(void *)g.hot.rows, (void *)g.hot.len, (void *)g.hot.cold_items, (void *)g.hot.cold_split,
                    (void *)g.hot.w3})
        dfree(p);
    g.hot = HotSet{};
    free_batch_state(g.batch);
    dfree(g.deg_u);
    g.deg_u = nullptr;
    dfree(g.u_new);
    g.u_new = nullptr;
    g.u_new_host.clear();
    free_query_state(g.q);
    for (void *p : {(void *)g.inv_b, g.tk_scratch})
        dfree(p);
    g.inv_b = nullptr;
    g.tk_scratch = nullptr;
}

}  // namespace ahpp
