// The hot rows of the batched V / attribute half-step as a dense product on
// the matrix cores.
//
// For the (at most 128) longest back rows x_h -- the most popular attributes
// and V nodes, 2% to 40% dense over U on the benchmark graphs -- the sums
//     S[h][q] = sum_u w'(u, x_h) Q[u][q]
// over every U node u and the queries q of a tile form a product of a
// 128 x n_U weight block and the tile's bf16 transport rows (Q, n_U x 256).
// The weights are stored dense, each split into three bfloat16 parts
// w' = w1 + w2 + w3 (rounded to nearest in turn, which keeps about 27 of its
// bits, more than float32's 24), so every product w_i * Q is exact in
// float32 and v_mfma_f32_32x32x16_bf16 accumulates them in float32.  U is
// cut into chunks of kc rows; workgroup (chunk c, tile t) writes the
// 128 x 256 partial of its chunk, and the reduction adds the partials in
// chunk order, so results are deterministic.
//
// Operand layouts of v_mfma_f32_32x32x16_bf16 (checked on the device):
// A[m][k] sits at lane m + 32 (k / 8), element k % 8; B[k][n] at lane
// n + 32 (k / 8), element k % 8; C[m][n] at lane n + 32 ((m / 4) % 2),
// element 4 (m / 8) + m % 4.  The weights are stored in that A order
// (1 KB per 32 rows x 16 columns, one 16-byte load per lane); the transport
// rows are staged through LDS transposed ([query][u], 16 bytes per lane read;
// each thread transposes a 4-row x 8-query block in registers and writes 8
// bytes per query).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "ahpp_internal.h"

namespace ahpp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kHB = 32;                       // hot rows per MFMA block (M)
constexpr int kHBlocks = kHotMax / kHB;       // 4: one per wave
constexpr int kKS = 16;                       // K of one MFMA
constexpr int kStageU = 32;                   // U rows per LDS stage (two K-steps)
constexpr int kQBlocks = kTileQ / 32;         // 8 query blocks (N) per tile
constexpr int kQsStride = 40;                 // bf16 per staged query row: 32 used + 8 pad (80 B)
constexpr int kDenseThreads = kHBlocks * kWave;
constexpr int kFragElems = 64 * 8;            // bf16 per A fragment (1 KB)
static_assert(kTileQ == 256, "the staging assignment assumes 256 queries per tile");
static_assert(kHotMax == 128, "four 32-row MFMA blocks");

// Nearest bfloat16 of a finite float (bits), ties to even.
__device__ __forceinline__ uint32_t bf16_rn_bits(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }

// Offset (bf16 elements) of weight (h, u) of part p in the A-fragment order.
__device__ __forceinline__ int64_t w3_offset(int p, int64_t n_ks, int h, int64_t u) {
    const int64_t ks = u / kKS;
    const int kk = (int)(u % kKS);
    const int lane = (h % kHB) + 32 * (kk / 8);
    return ((((int64_t)p * n_ks + ks) * kHBlocks + h / kHB) * 64 + lane) * 8 + kk % 8;
}

// One workgroup per hot row: each run of entries with the same U column (a
// repeated pair) is summed in order, split into three bf16 parts and stored.
__global__ void __launch_bounds__(kBlock) k_hot_w3(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                   const float *__restrict__ w, const int32_t *__restrict__ rows,
                                                   int64_t n_ks, uint16_t *w3) {
    const int h = blockIdx.x;
    const int32_t x = rows[h];
    const int64_t b = off[x], e = off[x + 1];
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const int32_t u = col[i];
        if (i > b && col[i - 1] == u) continue;
        float s = w[i];
        for (int64_t j = i + 1; j < e && col[j] == u; ++j) s += w[j];
        const uint32_t h1 = bf16_rn_bits(s);
        const float r1 = s - bf16_to_f(h1);
        const uint32_t h2 = bf16_rn_bits(r1);
        const float r2 = r1 - bf16_to_f(h2);
        const uint32_t h3 = bf16_rn_bits(r2);
        w3[w3_offset(0, n_ks, h, u)] = (uint16_t)h1;
        w3[w3_offset(1, n_ks, h, u)] = (uint16_t)h2;
        w3[w3_offset(2, n_ks, h, u)] = (uint16_t)h3;
    }
}

struct DenseArgs {
    const uint16_t *q;      // transport rows Q (tile 0), [n_u][kTileQ]
    int64_t q_stride;       // elements per tile
    const TileCtl *ctl;
    const uint16_t *w3;     // [3][n_ks][kHBlocks][64][8]
    int64_t n_ks;           // K-steps of 16 U rows per part
    int64_t kc;             // U rows per chunk (a multiple of kStageU)
    int64_t n_u;
    int n_hot, n_chunks, nt;
    float *part;            // partials (tile 0), [n_chunks][n_hot][kTileQ]
    int64_t part_stride;
};

// Workgroup c * nt + t: chunk c of tile t (the tiles of a chunk run next to
// each other, so its weights are read from HBM about once).  Wave w owns hot
// rows 32w .. 32w + 31 and all 256 queries of the tile: eight 32 x 32
// float32 accumulators.  Each stage stages 32 U rows of Q, transposed and
// with stopped queries zeroed, in LDS (double-buffered, one barrier per
// stage), and runs 2 K-steps x 3 weight parts x 8 query blocks of MFMA.
__global__ void __launch_bounds__(kDenseThreads) kb_hot_dense(DenseArgs a) {
    __shared__ __align__(16) uint16_t qs[2][kTileQ * kQsStride];
    const int c = blockIdx.x / a.nt, t = blockIdx.x % a.nt;
    const TileCtl &tc = a.ctl[t];
    if (tc.all_done) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const uint16_t *qt = a.q + t * a.q_stride;
    // Staging role: U rows 4 ub .. 4 ub + 3 of each stage and queries
    // 8 qg .. 8 qg + 7.  A thread loads its four 16-byte row pieces, zeroes
    // the stopped queries, transposes the 4 x 8 block in registers and
    // writes 8 bytes (4 U rows) per query.
    const int ub = tid & 7, qg = tid >> 3;
    u32x4 lm;  // 16-bit lane masks of the thread's 8 queries: all ones where the query runs
#pragma unroll
    for (int d = 0; d < 4; ++d)
        lm[d] = (tc.q[8 * qg + 2 * d].theta != FLT_MAX ? 0x0000FFFFu : 0u) |
                (tc.q[8 * qg + 2 * d + 1].theta != FLT_MAX ? 0xFFFF0000u : 0u);
    const int64_t u_begin = (int64_t)c * a.kc;
    const int n_stage = (int)(a.kc / kStageU);
    const int64_t ks_begin = u_begin / kKS;
    u32x4 stg[4];
    auto load_stage = [&](int st) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t u = u_begin + (int64_t)st * kStageU + 4 * ub + i;
            stg[i] = u < a.n_u ? __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(qt + u * kTileQ + 8 * qg))
                               : u32x4{0u, 0u, 0u, 0u};
        }
    };
    auto write_stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) stg[i] &= lm;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // query q is bytes 0-1 (q even) or 2-3 (q odd) of word q / 2 of
            // each row piece; lo packs rows 0 and 1, hi rows 2 and 3
            const uint32_t sel = (q & 1) ? 0x07060302u : 0x05040100u;
            const uint32_t lo = __builtin_amdgcn_perm(stg[1][q / 2], stg[0][q / 2], sel);
            const uint32_t hi = __builtin_amdgcn_perm(stg[3][q / 2], stg[2][q / 2], sel);
            *reinterpret_cast<uint2 *>(&qs[buf][(8 * qg + q) * kQsStride + 4 * ub]) = make_uint2(lo, hi);
        }
    };
    bf16x8 af[2][3], an[2][3];
    auto load_a = [&](int st, bf16x8 (&dst)[2][3]) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int64_t ks = ks_begin + (int64_t)st * 2 + s;
                const u32x4 raw = *reinterpret_cast<const u32x4 *>(
                    a.w3 + (((int64_t)p * a.n_ks + ks) * kHBlocks + wave) * kFragElems + lane * 8);
                dst[s][p] = __builtin_bit_cast(bf16x8, raw);
            }
    };
    f32x16 acc[kQBlocks];
#pragma unroll
    for (int qb = 0; qb < kQBlocks; ++qb) acc[qb] = f32x16{};
    load_stage(0);
    load_a(0, af);
    write_stage(0);
    __syncthreads();
    for (int st = 0; st < n_stage; ++st) {
        const int buf = st & 1;
        const bool more = st + 1 < n_stage;
        if (more) {
            load_stage(st + 1);
            load_a(st + 1, an);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 bf[kQBlocks];
#pragma unroll
            for (int qb = 0; qb < kQBlocks; ++qb) {
                const u32x4 raw = *reinterpret_cast<const u32x4 *>(
                    &qs[buf][(qb * 32 + (lane & 31)) * kQsStride + s * kKS + (lane >> 5) * 8]);
                bf[qb] = __builtin_bit_cast(bf16x8, raw);
            }
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int qb = 0; qb < kQBlocks; ++qb)
                    acc[qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[s][p], bf[qb], acc[qb], 0, 0, 0);
        }
        if (more) write_stage(buf ^ 1);
        __syncthreads();
        if (more) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int p = 0; p < 3; ++p) af[s][p] = an[s][p];
        }
    }
    float *pt = a.part + t * a.part_stride + (int64_t)c * a.n_hot * kTileQ;
#pragma unroll
    for (int qb = 0; qb < kQBlocks; ++qb)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int h = wave * kHB + 8 * (j / 4) + 4 * (lane >> 5) + (j % 4);
            if (h < a.n_hot) pt[(int64_t)h * kTileQ + qb * 32 + (lane & 31)] = acc[qb][j];
        }
}

}  // namespace

void dense_chunking(int64_t n_u, int64_t *kc, int64_t *n_chunks) {
    int64_t c = (n_u + kDenseChunks - 1) / kDenseChunks;
    c = (c + kStageU - 1) / kStageU * kStageU;
    *kc = std::max<int64_t>(c, kStageU);
    *n_chunks = std::max<int64_t>(1, (n_u + *kc - 1) / *kc);
}

namespace {
// K-steps of the weight block: U padded to whole chunks (zero weights).
int64_t dense_block_ks(int64_t n_u) {
    int64_t kc, n_chunks;
    dense_chunking(n_u, &kc, &n_chunks);
    return n_chunks * kc / kKS;
}
}  // namespace

size_t hot_dense_bytes(const Graph &g) {
    return (size_t)3 * (size_t)dense_block_ks(g.n_u) * kHBlocks * kFragElems * 2;
}

void build_hot_dense(Graph &g, hipStream_t s) {
    HotSet &h = g.hot;
    if (h.n <= 0 || g.n_u <= 0) return;
    const int64_t n_ks = dense_block_ks(g.n_u);
    const size_t bytes = hot_dense_bytes(g);
    h.w3 = (uint16_t *)dev_alloc(g, bytes, "dense hot weights");
    check_hip(hipMemsetAsync(h.w3, 0, bytes, s), "dense hot weights");
    hipLaunchKernelGGL(k_hot_w3, dim3((unsigned)h.n), dim3(kBlock), 0, s, (const int64_t *)g.back.off,
                       (const int32_t *)g.back.col, (const float *)g.back.w, (const int32_t *)h.rows, n_ks, h.w3);
    check_hip(hipGetLastError(), "dense hot weights launch");
    h.dense_ks = n_ks;
}

void launch_hot_dense(const Graph &g, const uint16_t *q, int64_t q_stride, const TileCtl *ctl, int nt, float *part,
                      int64_t part_stride, hipStream_t s) {
    const HotSet &h = g.hot;
    int64_t kc, n_chunks;
    dense_chunking(g.n_u, &kc, &n_chunks);
    DenseArgs a{q, q_stride, ctl, h.w3, h.dense_ks, kc, g.n_u, h.n, (int)n_chunks, nt, part, part_stride};
    hipLaunchKernelGGL(kb_hot_dense, dim3((unsigned)(n_chunks * nt)), dim3(kDenseThreads), 0, s, a);
}

}  // namespace ahpp
