// Batched AHPP queries on gfx950: the rounds of Algorithm 4 for many sources
// at once, sharing every pass over the edge lists.
//
// Queries are independent (each has its own residues, reserves, eps_f,
// threshold, phase and stop rule), so a batch is a set of tiles of kTileQ
// queries.  A tile's vectors are stored node-major: node x owns the kTileQ
// values [x][0..kTileQ) (1 KB of float32 state, 512 bytes of bfloat16
// transport).  A round is the same pair of pull-form gathers as the
// single-query path (z = inv_b * W'^T thr(r), then r <- keep(r) + W z with
// the reserve update), but every CSR entry is read once per tile and drives
// one contiguous 512-byte gather of all the tile's queries.  Row bookkeeping
// is wave-uniform (scalar), columns and weights arrive through scalar loads,
// and each wave keeps 8 KB of gathers in flight.  The forward gather reads
// two entries per 16-byte lane load (one per half-wave): gathers that hit
// L2 are bound by the number of load instructions (about 28 G wave loads/s
// on MI355X whatever their width), those that miss by bytes (about 7.5 TB/s
// for random rows), and half of the forward gathers hit.
//
// A query that has stopped keeps threshold +inf: it pushes nothing, so its
// state no longer changes while the rest of its tile runs on.
//
// Transport precision.  Residues and reserves stay float32, but what one
// half-step hands to the other moves as bfloat16 rounded toward zero (the top
// 16 bits of the float), with the exact remainder kept where it was:
//   * a U node that clears the threshold (r(u) > theta, compared in float32
//     as Algorithm 4 does) pushes q(u) = rz16(r(u)) <= r(u) and keeps
//     r(u) - q(u) (exact in float32) as residue.  The forward half-step of
//     one round writes Q(u) = r(u) > theta ? rz16(r(u)) : 0 for the next,
//     which the back gather reads; the next forward epilogue recomputes the
//     same value from r(u) and that round's theta (theta_q), so both halves
//     push the same amount;
//   * a V / attribute row x hands on zh(x) = rz16(z(x)) and keeps the carry
//     c(x) = z(x) - zh(x) for its next round; the forward gather reads the
//     bf16 table ZH.
// A push of any amount up to the residue keeps Lemma 2's invariant once the
// carries count as residues at their rows (they are mass on its way from V /
// the attributes to U), so with r'(u) = r(u) + sum_x w(u,x) c(x), the residue
// a push of every carry would leave, pi - pi_hat = sum_j r'(j) pi(j, .).
// Since c(x) < 2^-7 zh(x), r'(u) <= r(u) + 2^-7 s(u) with s(u) the sum this
// round pulled in, and the stop rule tests that bound against eps_f, so
// Theorem 2's eps holds as stated.  The random row gathers, which set the
// time of a round, move 512 bytes per tile row instead of 1 KB.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>

#include "ahpp_internal.h"
#include "dev_util.h"

namespace ahpp {

namespace {

static_assert(kVec == 4, "the gathers move 4 bf16 values (8 bytes) per lane and entry");
static_assert(kTileQ <= kBlock, "one workgroup thread per tile query");

constexpr int kWavesPerBlock = kBlock / kWave;
// CSR entries per group of loads issued before the first is used: one entry
// per 8-byte lane load (back gather), two per 16-byte lane load (forward).
constexpr int kGroupSingle = 16;
constexpr int kGroupPair = 16;
static_assert(kGroupSingle <= kCsrPad + 1 && kGroupPair <= kCsrPad + 1 && kGroupPair % 2 == 0,
              "a group may read up to group - 1 entries past a row (the CSR padding)");
constexpr int kMaskWords = kTileQ / 64;
enum BMode { kBBack = 0, kBFwd = 1 };

// The kVec queries of one lane.
struct QV {
    float v[kVec];
};

__device__ __forceinline__ QV qv_zero() {
    QV a;
#pragma unroll
    for (int j = 0; j < kVec; ++j) a.v[j] = 0.0f;
    return a;
}

__device__ __forceinline__ QV qv_load(const float *p) {
    QV a;
    if constexpr (kVec == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        a.v[0] = t.x;
        a.v[kVec > 1 ? 1 : 0] = t.y;
        a.v[kVec > 2 ? 2 : 0] = t.z;
        a.v[kVec > 3 ? 3 : 0] = t.w;
    } else if constexpr (kVec == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        a.v[0] = t.x;
        a.v[kVec - 1] = t.y;
    } else {
        a.v[0] = p[0];
    }
    return a;
}

__device__ __forceinline__ void qv_store(float *p, const QV &a) {
    if constexpr (kVec == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(a.v[0], a.v[kVec > 1 ? 1 : 0], a.v[kVec > 2 ? 2 : 0],
                                                     a.v[kVec > 3 ? 3 : 0]);
    } else if constexpr (kVec == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(a.v[0], a.v[kVec - 1]);
    } else {
        p[0] = a.v[0];
    }
}

// Transport values: bfloat16 rounded toward zero, i.e. the top 16 bits of a
// float; kVec of them per lane (8 bytes).
constexpr float kCarryBound = 0.0078125f;  // 2^-7: carry < kCarryBound * rz16(value)

__device__ __forceinline__ float rz16(float v) { return __uint_as_float(__float_as_uint(v) & 0xFFFF0000u); }

// Streaming (non-temporal) access to per-row state that no other wave of
// the launch reads again, so it does not push gathered rows out of L2
// (measured: 464 -> 481 queries/s on the bench batch).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ QV qv_load_nt(const float *p) {
    const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    QV a;
    a.v[0] = t.x; a.v[1] = t.y; a.v[2] = t.z; a.v[3] = t.w;
    return a;
}
__device__ __forceinline__ void qv_store_nt(float *p, const QV &a) {
    nt_f4 t;
    t.x = a.v[0]; t.y = a.v[1]; t.z = a.v[2]; t.w = a.v[3];
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4 *>(p));
}
__device__ __forceinline__ void qh_store_nt(uint16_t *p, const QV &a) {
    nt_u2 t;
    t.x = (__float_as_uint(a.v[0]) >> 16) | (__float_as_uint(a.v[1]) & 0xFFFF0000u);
    t.y = (__float_as_uint(a.v[2]) >> 16) | (__float_as_uint(a.v[3]) & 0xFFFF0000u);
    __builtin_nontemporal_store(t, reinterpret_cast<nt_u2 *>(p));
}

struct BArgs {
    const int64_t *__restrict__ off;
    const int32_t *__restrict__ col;
    const float *__restrict__ w;          // nullable (unit weights, fwd only)
    const WorkItem *__restrict__ items;
    int64_t n_items;
    const SplitRow *__restrict__ split;
    int64_t n_split;
    const uint16_t *x;     // gathered bf16 table (tile 0), rows of kTileQ: Q (kBBack) or ZH (kBFwd)
    float *y;              // written float rows (tile 0): carries (kBBack) or residues (kBFwd)
    uint16_t *yh;          // written bf16 rows (tile 0): ZH (kBBack) or Q (kBFwd)
    float *pi;             // reserves (tile 0), kBFwd
    const float *inv_b;    // kBBack row scale
    float *part;           // chunk partials (tile 0), [item][kTileQ]
    TileCtl *ctl;          // tile 0
    int64_t x_stride, y_stride, pi_stride, part_stride;  // elements per tile (y and yh share y_stride)
    float *blk_max;        // [tile][2][batch_cap][kTileQ] slot base of this launch
    unsigned long long *blk_np;  // [tile][5][batch_cap][kTileQ] slot base
    int64_t blk_stride_f, blk_stride_u;   // elements per tile
    float alpha;
};

__device__ __forceinline__ float readlane_f(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// A value the same in every lane, held in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The kVec queries of a lane in the gathers' epilogues: lane l < 32 takes
// queries 8l .. 8l+3 and lane l + 32 takes 8l+4 .. 8l+7, the halves that the
// two-entry loads leave in each lane (see run_entries).
__device__ __forceinline__ int lane_q0() {
    const int l = threadIdx.x & 63;
    return 8 * (l & 31) + 4 * (l >> 5);
}
__device__ __forceinline__ int64_t lane_col() { return (int64_t)lane_q0(); }

// Per-lane epilogues over the lane's kVec queries.
template <int kMode>
struct BEpi;

template <>
struct BEpi<kBBack> {
    struct Pre {
        float scale;
        QV c;  // carries of the row
    };
    float *c;
    uint16_t *zh;
    QV theta;
    unsigned long long np[kVec];
    float mx[kVec];
    __device__ Pre pre(int64_t row, float scale) const { return Pre{scale, qv_load_nt(c + row * kTileQ + lane_col())}; }
    // z = carry + inv_b * sum; hands on zh = rz16(z), keeps z - zh.  A
    // stopped query (threshold +inf) hands on nothing and keeps its carries.
    __device__ void full(int64_t row, const QV &s, const Pre &p, int64_t len) {
        const int64_t i = row * kTileQ + lane_col();
        QV nc, h;
#pragma unroll
        for (int j = 0; j < kVec; ++j) {
            const float v = p.c.v[j] + p.scale * s.v[j];
            const bool live = theta.v[j] != FLT_MAX;
            h.v[j] = live ? rz16(v) : 0.0f;
            nc.v[j] = live ? v - h.v[j] : p.c.v[j];
            if (live && v > 0.0f) np[j] += (unsigned long long)len;
        }
        qv_store_nt(c + i, nc);
        qh_store_nt(zh + i, h);
    }
};

template <>
struct BEpi<kBFwd> {
    struct Pre {
        QV r, pi;
    };
    float *r;
    float *pi;
    uint16_t *q;
    QV theta;
    QV theta_q;
    float alpha;
    unsigned long long np[kVec];
    float mx[kVec];
    __device__ Pre pre(int64_t row, float) const {
        const int64_t i = row * kTileQ + lane_col();
        return Pre{qv_load_nt(r + i), qv_load_nt(pi + i)};
    }
    // u pushed in the back half-step the Q value of its residue (rz16(r) if r
    // cleared the threshold Q was cut with, else 0) and keeps the exact rest;
    // the next round's Q is cut with this round's threshold.  The stop
    // statistic bounds the residue left once the carries are pushed too.
    __device__ void full(int64_t row, const QV &s, const Pre &p, int64_t len) {
        const int64_t i = row * kTileQ + lane_col();
        QV nr, np_, nq;
#pragma unroll
        for (int j = 0; j < kVec; ++j) {
            const bool live = theta.v[j] != FLT_MAX;
            const float qv = live && p.r.v[j] > theta_q.v[j] ? rz16(p.r.v[j]) : 0.0f;
            const bool pushed = qv > 0.0f;
            np_.v[j] = pushed ? p.pi.v[j] + alpha * qv : p.pi.v[j];
            if (pushed) np[j] += (unsigned long long)len;
            nr.v[j] = (p.r.v[j] - qv) + s.v[j];
            nq.v[j] = nr.v[j] > theta.v[j] ? nr.v[j] : 0.0f;
            mx[j] = fmaxf(mx[j], nr.v[j] + kCarryBound * s.v[j]);
        }
        qv_store_nt(pi + i, np_);
        qv_store_nt(r + i, nr);
        qh_store_nt(q + i, nq);
    }
};

// Sum over entries [e0, e0 + ne) of w * x[col] for every query of the tile,
// flushing each completed row of [r0, r0 + n_rows) through the epilogue.
// Row ends are relative to e0; rows may be empty.  r0, n_rows, e0, ne and
// every row end are the same in all lanes (the caller makes them so).
//
// One 16-byte load per lane fetches two entries: lanes 0-31 read the 512-byte
// transport row of entry k (8 queries each) and lanes 32-63 that of entry
// k + 1, so a wave issues one load per two entries and keeps each lane's 8
// partial sums.  At a row end the two halves are added with one lane swap
// (v_permlane32_swap) per pair of sums, which leaves every lane the totals of
// its 4 epilogue queries (lane_q0).  When a row ends between the two entries
// of a load, the lower half is added first, the row flushed, then the upper
// half added for the next row.  Columns and weights come a group at a time
// through scalar loads; slots past the last entry read the entries that
// follow (the CSR's zero padding at its end) and add them with weight 0.  A
// stopped query's sums are computed like the others and discarded by the
// epilogue.
template <bool kUnit, int kMode, bool kPaired, class RowEnd, class RowScale>
__device__ __forceinline__ void run_entries(const int32_t *__restrict__ col, const float *__restrict__ wt,
                                            const uint16_t *__restrict__ xt, int64_t r0, int n_rows, int64_t e0,
                                            int ne, BEpi<kMode> &epi, RowEnd row_end, RowScale row_scale,
                                            QV *acc_out) {
    using Pre = typename BEpi<kMode>::Pre;
    const int lane = threadIdx.x & (kWave - 1);
    const bool upper = lane >= 32;
    // Each half picks its entry's column and weight from the scalar pair
    // with a lane mask (bit operations, so the pair stays in registers).
    const uint32_t umask = upper ? ~0u : 0u;
    auto pick = [&](uint32_t lo, uint32_t hi) { return lo ^ ((lo ^ hi) & umask); };
    const char *xl = reinterpret_cast<const char *>(xt) + (uint32_t)(lane & 31) * 16u;
    int j = 0, rstart = 0;
    int rend = n_rows > 0 ? row_end(0) : INT_MAX;
    Pre pre = epi.pre(r0, n_rows > 0 ? row_scale(0) : 0.0f);
    float acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
    // The 4 totals of this lane's epilogue queries.
    auto totals = [&]() {
        QV s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[q]), __float_as_uint(acc[q + 4]),
                                                             false, false);
            s.v[q] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
        return s;
    };
    // Flushes every row that ends at entry position e.
    auto flush_at = [&](int e) {
        while (e == rend) {
            epi.full(r0 + j, totals(), pre, rend - rstart);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
            rstart = rend;
            ++j;
            if (j < n_rows) {
                rend = row_end(j);
                pre = epi.pre(r0 + j, row_scale(j));
            } else {
                rend = INT_MAX;
            }
        }
    };
    flush_at(0);
    if constexpr (!kPaired) {
        // One entry per load: each lane reads its 4 epilogue queries (8 bytes)
        // of the entry's row, and its sums need no combining.
        const char *xq = reinterpret_cast<const char *>(xt) + (uint32_t)lane_q0() * 2u;
        QV a4 = qv_zero();
        auto flush1 = [&](int e) {
            while (e == rend) {
                epi.full(r0 + j, a4, pre, rend - rstart);
                a4 = qv_zero();
                rstart = rend;
                ++j;
                if (j < n_rows) {
                    rend = row_end(j);
                    pre = epi.pre(r0 + j, row_scale(j));
                } else {
                    rend = INT_MAX;
                }
            }
        };
        for (int k0 = 0; k0 < ne; k0 += kGroupSingle) {
            int32_t cn[kGroupSingle];
            float wk[kGroupSingle];
#pragma unroll
            for (int u = 0; u < kGroupSingle; ++u) cn[u] = col[e0 + k0 + u];
#pragma unroll
            for (int u = 0; u < kGroupSingle; ++u) wk[u] = kUnit ? 1.0f : wt[e0 + k0 + u];
            uint2 v[kGroupSingle];
#pragma unroll
            for (int u = 0; u < kGroupSingle; ++u)
                v[u] = *reinterpret_cast<const uint2 *>(xq + (uint64_t)(uint32_t)cn[u] * (kTileQ * 2));
            if (ne - k0 < kGroupSingle) {
#pragma unroll
                for (int u = 0; u < kGroupSingle; ++u)
                    if (u >= ne - k0) wk[u] = 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kGroupSingle; ++u) {
                const float xu[4] = {__uint_as_float(v[u].x << 16), __uint_as_float(v[u].x & 0xFFFF0000u),
                                     __uint_as_float(v[u].y << 16), __uint_as_float(v[u].y & 0xFFFF0000u)};
#pragma unroll
                for (int q = 0; q < 4; ++q) a4.v[q] += wk[u] * xu[q];
                flush1(k0 + u + 1);
            }
        }
        if (acc_out) *acc_out = a4;
        return;
    }
    for (int k0 = 0; k0 < ne; k0 += kGroupPair) {
        int32_t cn[kGroupPair];
        float wk[kGroupPair];
#pragma unroll
        for (int u = 0; u < kGroupPair; ++u) cn[u] = col[e0 + k0 + u];
#pragma unroll
        for (int u = 0; u < kGroupPair; ++u) wk[u] = kUnit ? 1.0f : wt[e0 + k0 + u];
        uint4 v[kGroupPair / 2];  // packed transport values, unpacked when added
#pragma unroll
        for (int p = 0; p < kGroupPair / 2; ++p) {
            const uint32_t c = pick((uint32_t)cn[2 * p], (uint32_t)cn[2 * p + 1]);
            v[p] = *reinterpret_cast<const uint4 *>(xl + (uint64_t)c * (kTileQ * 2));
        }
        if (ne - k0 < kGroupPair) {
#pragma unroll
            for (int u = 0; u < kGroupPair; ++u)
                if (u >= ne - k0) wk[u] = 0.0f;
        }
#pragma unroll
        for (int p = 0; p < kGroupPair / 2; ++p) {
            const uint32_t b[4] = {v[p].x, v[p].y, v[p].z, v[p].w};
            float x[8];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                x[2 * h] = __uint_as_float(b[h] << 16);
                x[2 * h + 1] = __uint_as_float(b[h] & 0xFFFF0000u);
            }
            const int e_lo = k0 + 2 * p + 1;
            if (rend != e_lo) {
                // Both entries belong to the current row.
                const float w = __uint_as_float(pick(__float_as_uint(wk[2 * p]), __float_as_uint(wk[2 * p + 1])));
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += w * x[q];
            } else {
                const float wl = __uint_as_float(pick(__float_as_uint(wk[2 * p]), 0u));
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += wl * x[q];
                flush_at(e_lo);
                const float wu = __uint_as_float(pick(0u, __float_as_uint(wk[2 * p + 1])));
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += wu * x[q];
            }
            flush_at(e_lo + 1);
        }
    }
    if (acc_out) *acc_out = totals();
}

template <int kMode>
__device__ __forceinline__ BEpi<kMode> make_bepi(const BArgs &a, int t, const QV &theta) {
    BEpi<kMode> e;
    if constexpr (kMode == kBBack) {
        e.c = a.y + t * a.y_stride;
        e.zh = a.yh + t * a.y_stride;
    } else {
        e.r = a.y + t * a.y_stride;
        e.q = a.yh + t * a.y_stride;
        e.pi = a.pi + t * a.pi_stride;
        e.alpha = a.alpha;
    }
    e.theta = theta;
    if constexpr (kMode == kBFwd) {
        const int q0 = lane_q0();
#pragma unroll
        for (int j = 0; j < kVec; ++j) e.theta_q.v[j] = a.ctl[t].q[q0 + j].theta_q;
    }
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        e.np[j] = 0;
        e.mx[j] = 0.0f;
    }
    return e;
}

__device__ __forceinline__ QV lane_theta(const TileCtl &tc) {
    QV th;
    const int q0 = lane_q0();
#pragma unroll
    for (int j = 0; j < kVec; ++j) th.v[j] = tc.q[q0 + j].theta;
    return th;
}

// Per-workgroup max and n_p of every query of the tile, one slot per query.
template <int kMode>
__device__ __forceinline__ void bflush(const BArgs &a, int t, int j, BEpi<kMode> &epi) {
    __shared__ float smx[kWavesPerBlock][kTileQ];
    __shared__ unsigned long long snp[kWavesPerBlock][kTileQ];
    const int q0 = lane_q0(), wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        smx[wid][q0 + j] = epi.mx[j];
        snp[wid][q0 + j] = epi.np[j];
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < kTileQ) {
        float m = smx[0][q];
        unsigned long long n = snp[0][q];
#pragma unroll
        for (int i = 1; i < kWavesPerBlock; ++i) {
            m = fmaxf(m, smx[i][q]);
            n += snp[i][q];
        }
        const int64_t o = (int64_t)j * kTileQ + q;
        if (a.blk_max) a.blk_max[t * a.blk_stride_f + o] = m;
        if (a.blk_np) a.blk_np[t * a.blk_stride_u + o] = n;
    }
}

template <bool kUnit, int kMode>
__global__ void __launch_bounds__(kBlock, 4) kb_gather(BArgs a, const int32_t *__restrict__ col,
                                                    const float *__restrict__ wt) {
    const int t = blockIdx.y, wg = blockIdx.x;
    const TileCtl &tc = a.ctl[t];
    if (tc.all_done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint16_t *xt = a.x + t * a.x_stride;
    float *part = a.part + t * a.part_stride;
    BEpi<kMode> epi = make_bepi<kMode>(a, t, lane_theta(tc));
    const int64_t wave0 = (int64_t)wg * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t it = wave0; it < a.n_items; it += stride) {
        WorkItem item = a.items[it];
        item.row = __builtin_amdgcn_readfirstlane(item.row);
        item.n = __builtin_amdgcn_readfirstlane(item.n);
        if (item.n > 0) {
            const int64_t r0 = item.row;
            const int n = item.n;
            const int64_t e0 = uniform64(a.off[r0]);
            const int ne = __builtin_amdgcn_readfirstlane((int)(a.off[r0 + n] - e0));
            // Row ends (relative to e0) and row scales, one row per lane.
            int end0 = INT_MAX, end1 = INT_MAX;
            float sc0 = 0.0f, sc1 = 0.0f;
            if (lane < n) end0 = (int)(a.off[r0 + lane + 1] - e0);
            if (lane + kWave < n) end1 = (int)(a.off[r0 + lane + kWave + 1] - e0);
            if constexpr (kMode == kBBack) {
                if (lane < n) sc0 = a.inv_b[r0 + lane];
                if (lane + kWave < n) sc1 = a.inv_b[r0 + lane + kWave];
            }
            auto row_end = [&](int jj) {
                return jj < kWave ? __builtin_amdgcn_readlane(end0, jj) : __builtin_amdgcn_readlane(end1, jj - kWave);
            };
            auto row_scale = [&](int jj) { return jj < kWave ? readlane_f(sc0, jj) : readlane_f(sc1, jj - kWave); };
            run_entries<kUnit, kMode, kMode == kBFwd>(col, wt, xt, r0, n, e0, ne, epi, row_end, row_scale, nullptr);
        } else {
            const int64_t row = item.row;
            const int64_t rb = uniform64(a.off[row]), re = uniform64(a.off[row + 1]);
            const int64_t e0 = rb + (int64_t)(-item.n) * kItemEdges;
            const int ne = (int)(re - e0 < kItemEdges ? re - e0 : kItemEdges);
            const bool whole = re - rb <= kItemEdges;
            float scale = 0.0f;
            if constexpr (kMode == kBBack) scale = a.inv_b[row];
            auto row_end = [&](int) { return whole ? ne : INT_MAX; };
            auto row_scale = [&](int) { return scale; };
            QV acc;
            run_entries<kUnit, kMode, kMode == kBFwd>(col, wt, xt, row, whole ? 1 : 0, e0, ne, epi, row_end, row_scale,
                                                      &acc);
            if (!whole) qv_store(part + it * kTileQ + lane_col(), acc);
        }
    }
    bflush<kMode>(a, t, wg, epi);
}

// Rows cut into chunks: one wave per row adds its chunk sums per query.
template <int kMode>
__global__ void __launch_bounds__(kBlock) kb_fix(BArgs a) {
    const int t = blockIdx.y, wg = blockIdx.x;
    const TileCtl &tc = a.ctl[t];
    if (tc.all_done) return;
    const float *part = a.part + t * a.part_stride;
    BEpi<kMode> epi = make_bepi<kMode>(a, t, lane_theta(tc));
    const int64_t wave0 = (int64_t)wg * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t i = wave0; i < a.n_split; i += stride) {
        const SplitRow sr = a.split[i];
        QV s = qv_zero();
        const float *pr = part + (int64_t)sr.first_item * kTileQ + lane_col();
        int ch = 0;
        // Eight chunk loads in flight, added in chunk order.
        for (; ch + 8 <= sr.nch; ch += 8) {
            QV p[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) p[u] = qv_load(pr + (int64_t)(ch + u) * kTileQ);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int j = 0; j < kVec; ++j) s.v[j] += p[u].v[j];
        }
        for (; ch < sr.nch; ++ch) {
            const QV p = qv_load(pr + (int64_t)ch * kTileQ);
#pragma unroll
            for (int j = 0; j < kVec; ++j) s.v[j] += p.v[j];
        }
        const float scale = kMode == kBBack ? a.inv_b[sr.row] : 0.0f;
        epi.full(sr.row, s, epi.pre(sr.row, scale), a.off[sr.row + 1] - a.off[sr.row]);
    }
    bflush<kMode>(a, t, wg, epi);
}

// One workgroup per tile, one thread per query: max r and n_p from the
// partials, then the stop / switch rule of Algorithm 4 for every running query.
constexpr int kCtlSplit = 4;    // threads per query reducing the partials
constexpr int kCtlThreads = kCtlSplit * kTileQ;
constexpr int kCtlSlices = 32;  // workgroups per tile reducing the partials

// Workgroup (slice, tile), thread (part, q): max r and n_p of query q over
// the workgroup partials i with i % (kCtlSplit * kCtlSlices) ==
// slice * kCtlSplit + part; max and integer sums do not depend on the order.
__global__ void __launch_bounds__(kCtlThreads) kb_control_partials(
    const TileCtl *ctl, const float *blk_max, const unsigned long long *blk_np, int64_t stride_f, int64_t stride_u,
    int cap, int n_back, int n_back_fix, int n_fwd, int n_fwd_fix, int n_hot, float *red_max,
    unsigned long long *red_np) {
    __shared__ float s_max[kCtlSplit][kTileQ];
    __shared__ unsigned long long s_np[kCtlSplit][kTileQ];
    const int t = blockIdx.y;
    if (ctl[t].all_done) return;
    const int q = threadIdx.x % kTileQ, part = threadIdx.x / kTileQ;
    const int first = blockIdx.x * kCtlSplit + part, step = kCtlSplit * kCtlSlices;
    const float *bm = blk_max + t * stride_f;
    const unsigned long long *bn = blk_np + t * stride_u;
    float m = 0.0f;
    for (int i = first; i < n_fwd; i += step) m = fmaxf(m, bm[(int64_t)i * kTileQ + q]);
    for (int i = first; i < n_fwd_fix; i += step) m = fmaxf(m, bm[((int64_t)cap + i) * kTileQ + q]);
    unsigned long long np = 0;
    const int cnt[5] = {n_back, n_back_fix, n_fwd, n_fwd_fix, n_hot};
#pragma unroll
    for (int k = 0; k < 5; ++k)
        for (int i = first; i < cnt[k]; i += step) np += bn[((int64_t)k * cap + i) * kTileQ + q];
    s_max[part][q] = m;
    s_np[part][q] = np;
    __syncthreads();
    if (part == 0) {
#pragma unroll
        for (int i = 1; i < kCtlSplit; ++i) {
            m = fmaxf(m, s_max[i][q]);
            np += s_np[i][q];
        }
        const int64_t o = ((int64_t)t * kCtlSlices + blockIdx.x) * kTileQ + q;
        red_max[o] = m;
        red_np[o] = np;
    }
}

// One workgroup per tile, one thread per query: combines the slices, then
// the stop / switch rule of Algorithm 4 for every running query.
__global__ void __launch_bounds__(kTileQ) kb_control(TileCtl *ctl, const float *red_max,
                                                     const unsigned long long *red_np, Rule rule) {
    __shared__ int running_any[kTileQ / kWave];
    const int t = blockIdx.x;
    TileCtl &tc = ctl[t];
    if (tc.all_done) return;
    const int q = threadIdx.x;
    float m = 0.0f;
    unsigned long long np = 0;
#pragma unroll
    for (int i = 0; i < kCtlSlices; ++i) {
        const int64_t o = ((int64_t)t * kCtlSlices + i) * kTileQ + q;
        m = fmaxf(m, red_max[o]);
        np += red_np[o];
    }
    QueryCtl &c = tc.q[q];
    int done = c.done;
    if (!done) {
        c.theta_q = c.theta;  // the threshold this round's forward half-step cut Q with
        const unsigned long long n_p = c.n_p + np;
        const int iter = c.iter + 1;
        c.n_p = n_p;
        c.iter = iter;
        c.last_max = m;
        if (!(m > c.eps_f)) {
            done = 1;
            c.status = 1;
        } else if (iter >= c.max_iters) {
            done = 1;
            c.status = 2;
        } else if (c.phase == 1) {
            const double tt = (double)logf(m / c.eps_f) * (double)rule.inv_log;
            if ((double)n_p >= rule.budget_scale * (tt > 0.0 ? tt : 0.0)) {
                c.phase = 2;
                c.theta = 0.0f;
                c.switch_iter = iter;
            }
        }
        if (done) {
            c.done = 1;
            c.theta = FLT_MAX;
        }
    }
    const unsigned long long running = __ballot(!done);
    if ((q & 63) == 0) running_any[q >> 6] = running != 0ull;
    __syncthreads();
    if (q == 0) {
        int any = 0;
        for (int i = 0; i < kTileQ / kWave; ++i) any |= running_any[i];
        tc.all_done = any ? 0 : 1;
    }
}

// ---------------------------------------------------------------- hot rows

struct HotReduceArgs {
    const float *part;      // tile 0 partials
    int64_t part_stride;
    const int32_t *rows, *len;
    const float *inv_b;
    float *c;               // carries (tile 0)
    uint16_t *zh;           // bf16 transport rows ZH (tile 0)
    int64_t z_stride;
    unsigned long long *blk_np;  // n_p slot of this launch (tile 0)
    int64_t blk_stride_u;
    const TileCtl *ctl;
    int n_hot, n_chunks;
};

// One workgroup per (hot row, tile): z(x) = carry + inv_b(x) * (chunk
// partials added in chunk order), handed on as rz16(z) with the rest kept as
// carry (as the back gather's epilogue), and the row's entry count for the
// queries it pushes.
__global__ void __launch_bounds__(kBlock) kb_hot_reduce(HotReduceArgs a) {
    const int h = blockIdx.x, t = blockIdx.y;
    if (a.ctl[t].all_done) return;
    const int q = threadIdx.x;
    const float *pt = a.part + t * a.part_stride + (int64_t)h * kTileQ + q;
    const int64_t cs = (int64_t)a.n_hot * kTileQ;
    float s = 0.0f;
    int c = 0;
    for (; c + 8 <= a.n_chunks; c += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = pt[(c + j) * cs];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; c < a.n_chunks; ++c) s += pt[c * cs];
    const int32_t x = a.rows[h];
    const int64_t i = t * a.z_stride + (int64_t)x * kTileQ + q;
    const float c0 = a.c[i];
    const float v = c0 + a.inv_b[x] * s;
    const bool live = a.ctl[t].q[q].theta != FLT_MAX;
    const float h16 = live ? rz16(v) : 0.0f;
    a.c[i] = live ? v - h16 : c0;
    a.zh[i] = (uint16_t)(__float_as_uint(h16) >> 16);
    a.blk_np[t * a.blk_stride_u + (int64_t)h * kTileQ + q] = live && v > 0.0f ? (unsigned long long)a.len[h] : 0ull;
}

__global__ void kb_fill(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

constexpr uint16_t kOneBf16 = 0x3F80;  // 1.0f as bfloat16

struct InitQuery {
    int32_t source;
    float eps_f;
};

// One workgroup per tile, one thread per query: start query q of the tile
// (or leave the slot empty).
__global__ void __launch_bounds__(kTileQ) kb_init(TileCtl *ctl, float *r, uint16_t *qh, int64_t r_stride,
                                                  const InitQuery *qs, int64_t n_valid, int32_t max_iters) {
    __shared__ int running_any[kTileQ / kWave];
    const int t = blockIdx.x, q = threadIdx.x;
    const int64_t gq = (int64_t)t * kTileQ + q;
    QueryCtl &c = ctl[t].q[q];
    const bool live = gq < n_valid;
    const int32_t src = live ? qs[gq].source : -1;
    const float eps_f = live ? qs[gq].eps_f : 1.0f;
    const bool run = live && 1.0f > eps_f;
    if (live) {
        r[t * r_stride + (int64_t)src * kTileQ + q] = 1.0f;
        qh[t * r_stride + (int64_t)src * kTileQ + q] = kOneBf16;
    }
    c.theta = run ? eps_f : FLT_MAX;
    c.theta_q = 0.0f;  // Q holds the unit residue of the source, as cut with threshold 0
    c.pad = 0;
    c.eps_f = eps_f;
    c.done = run ? 0 : 1;
    c.phase = 1;
    c.iter = 0;
    c.switch_iter = -1;
    c.status = run ? 0 : 1;
    c.max_iters = max_iters;
    c.n_p = 0;
    c.last_max = live ? 1.0f : 0.0f;
    c.source = src;
    const unsigned long long running = __ballot(run);
    if ((q & 63) == 0) running_any[q >> 6] = running != 0ull;
    __syncthreads();
    if (q == 0) {
        int any = 0;
        for (int i = 0; i < kTileQ / kWave; ++i) any |= running_any[i];
        ctl[t].all_done = any ? 0 : 1;
    }
}

// Zeroes the residue, transport residue and reserve (U rows) and the carry
// (V / attribute rows) of the queries set in the tile's mask words
// (masks[t * kMaskWords + q / 64] bit q % 64).
__global__ void __launch_bounds__(kBlock) kb_clear_lanes(float *r, uint16_t *qh, float *pi, int64_t tile_u,
                                                         int64_t n_u, float *c, int64_t tile_x, int64_t n_x,
                                                         const unsigned long long *masks) {
    const int t = blockIdx.y;
    const unsigned long long *m = masks + (int64_t)t * kMaskWords;
    bool any = false;
#pragma unroll
    for (int i = 0; i < kMaskWords; ++i) any = any || m[i] != 0ull;
    if (!any) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    bool mine[kVec];
    bool some = false;
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        const int q = lane * kVec + j;
        mine[j] = (m[q >> 6] >> (q & 63)) & 1ull;
        some = some || mine[j];
    }
    if (!some) return;
    float *rt = r + t * tile_u, *pt = pi + t * tile_u, *ct = c + t * tile_x;
    uint16_t *qt = qh + t * tile_u;
    const int64_t step = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + wid; u < n_u; u += step) {
#pragma unroll
        for (int j = 0; j < kVec; ++j) {
            if (mine[j]) {
                const int64_t i = u * kTileQ + lane * kVec + j;
                rt[i] = 0.0f;
                pt[i] = 0.0f;
                qt[i] = 0;
            }
        }
    }
    for (int64_t x = (int64_t)blockIdx.x * kWavesPerBlock + wid; x < n_x; x += step) {
#pragma unroll
        for (int j = 0; j < kVec; ++j)
            if (mine[j]) ct[x * kTileQ + lane * kVec + j] = 0.0f;
    }
}

// Starts admitted queries: unit residue at the source and a fresh control.
__global__ void kb_admit(TileCtl *ctl, float *r, uint16_t *qh, int64_t tile_u, const AdmitReq *req, int n,
                         int32_t max_iters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const AdmitReq a = req[i];
    TileCtl &tc = ctl[a.tile];
    QueryCtl &c = tc.q[a.lane];
    const bool run = 1.0f > a.eps_f;
    r[a.tile * tile_u + (int64_t)a.source * kTileQ + a.lane] = 1.0f;
    qh[a.tile * tile_u + (int64_t)a.source * kTileQ + a.lane] = kOneBf16;
    c.theta = run ? a.eps_f : FLT_MAX;
    c.theta_q = 0.0f;
    c.pad = 0;
    c.eps_f = a.eps_f;
    c.done = run ? 0 : 1;
    c.phase = 1;
    c.iter = 0;
    c.switch_iter = -1;
    c.status = run ? 0 : 1;
    c.max_iters = max_iters;
    c.n_p = 0;
    c.last_max = 1.0f;
    c.source = a.source;
    if (run) tc.all_done = 0;
}

// Reads a 64-row block of one tile into LDS, rows in input order:
// tile[i][q] = pi[u_new[u0 + i]][q].
__device__ __forceinline__ void load_row_block(const float *pi, const int32_t *u_new, int64_t u0, int64_t n_u,
                                               float (*tile)[kTileQ + 1]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < kWave; i += kWavesPerBlock) {
        const int64_t u = u0 + i;
        const QV v = u < n_u ? qv_load(pi + (int64_t)u_new[u] * kTileQ + lane * kVec) : qv_zero();
#pragma unroll
        for (int j = 0; j < kVec; ++j) tile[i][lane * kVec + j] = v.v[j];
    }
    __syncthreads();
}

// out[j * n_u + u] = pi[u_new[u]][lanes[j]] for the j < n_sel selected
// queries of one tile (u in input order).
__global__ void __launch_bounds__(kBlock) kb_gather_lanes(const float *pi, const int32_t *u_new, int64_t n_u,
                                                          const int32_t *lanes, int n_sel, float *out) {
    __shared__ float tile[kWave][kTileQ + 1];
    const int64_t u0 = (int64_t)blockIdx.x * kWave;
    load_row_block(pi, u_new, u0, n_u, tile);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int j = wid; j < n_sel; j += kWavesPerBlock) {
        const int q = lanes[j];
        const int64_t u = u0 + lane;
        if (u < n_u) out[(int64_t)j * n_u + u] = tile[lane][q];
    }
}

// out[(t * kTileQ + q) * n_u + u] = pi[t][u_new[u]][q] for rows t * kTileQ + q
// < n_rows_valid (u in input order).
__global__ void __launch_bounds__(kBlock) kb_transpose(const float *pi, int64_t pi_stride, const int32_t *u_new,
                                                       int64_t n_u, float *out, int64_t n_rows_valid) {
    __shared__ float tile[kWave][kTileQ + 1];
    const int t = blockIdx.y;
    const int64_t u0 = (int64_t)blockIdx.x * kWave;
    load_row_block(pi + t * pi_stride, u_new, u0, n_u, tile);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int q = wid; q < kTileQ; q += kWavesPerBlock) {
        const int64_t row = (int64_t)t * kTileQ + q;
        const int64_t u = u0 + lane;
        if (row < n_rows_valid && u < n_u) out[row * n_u + u] = tile[lane][q];
    }
}

// Per-query sums of a tile vector: blk[t][block][q].
__global__ void __launch_bounds__(kBlock) kb_sums(const float *x, int64_t x_stride, int64_t n_u, double *blk) {
    __shared__ double s[kWavesPerBlock][kTileQ];
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const float *xt = x + t * x_stride;
    double acc[kVec];
#pragma unroll
    for (int j = 0; j < kVec; ++j) acc[j] = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + wid; u < n_u; u += (int64_t)gridDim.x * kWavesPerBlock) {
        const QV v = qv_load(xt + u * kTileQ + lane * kVec);
#pragma unroll
        for (int j = 0; j < kVec; ++j) acc[j] += (double)v.v[j];
    }
#pragma unroll
    for (int j = 0; j < kVec; ++j) s[wid][lane * kVec + j] = acc[j];
    __syncthreads();
    const int q = threadIdx.x;
    if (q < kTileQ) {
        double v = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) v += s[i][q];
        blk[((int64_t)t * gridDim.x + blockIdx.x) * kTileQ + q] = v;
    }
}

// Workgroups per tile of a batch gather launch are at most this many (the
// per-workgroup partial slots are sized for it): twice the single-query cap,
// so the tuner can try up to 8x the default share per tile.
int batch_cap(const Graph &g) { return 2 * g.grid_cap; }

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

struct BPlan {
    unsigned back, back_fix, fwd, fwd_fix;
};


// Workgroups per tile: enough waves to cover the items, at most the
// per-launch budget spread over the tiles in flight.
// The back schedule of the batched engine: every row, or only the cold rows
// when the graph has hot rows.
struct BackSched {
    const WorkItem *items;
    int64_t n_items;
    const SplitRow *split;
    int64_t n_split;
    int64_t nnz, rows;
};

BackSched back_sched(const Graph &g) {
    const HotSet &h = g.hot;
    if (h.n > 0) return BackSched{h.cold_items, h.n_cold_items, h.cold_split, h.n_cold_split, h.cold_nnz, h.cold_rows};
    return BackSched{g.back.items, g.back.n_items, g.back.split, g.back.n_split, g.back.nnz, g.back.n_rows};
}

BPlan bplan(const Graph &g, int nt) {
    const int cap = std::min(batch_cap(g), std::max(64, g.tuned_wg_mult * g.grid_cap / std::max(nt, 1)));
    const BackSched bs = back_sched(g);
    BPlan p;
    p.back = bs.n_items ? capped(bs.n_items, kWavesPerBlock, cap) : 0;
    p.back_fix = bs.n_split ? capped(bs.n_split, kWavesPerBlock, cap) : 0;
    p.fwd = capped(g.fwd.n_items, kWavesPerBlock, cap);
    p.fwd_fix = g.fwd.n_split ? capped(g.fwd.n_split, kWavesPerBlock, cap) : 0;
    return p;
}

}  // namespace

void free_batch_state(BatchState &b) {
    for (auto &e : b.round_graphs) (void)hipGraphExecDestroy(e.second);
    for (void *p : {(void *)b.r, (void *)b.pi, (void *)b.q, (void *)b.c, (void *)b.zh, (void *)b.part, (void *)b.ctl,
                    (void *)b.blk_max,
                    (void *)b.blk_np, (void *)b.red_max, (void *)b.red_np, (void *)b.hot_part, (void *)b.out,
                    (void *)b.sums})
        dfree(p);
    b = BatchState{};
}

// Chunks of the hot-row partials (the dense pass's U chunks).
int64_t hot_chunks(const Graph &g) {
    int64_t kc, n_chunks;
    dense_chunking(g.n_u, &kc, &n_chunks);
    return n_chunks;
}

int64_t batch_tile_bytes(const Graph &g, bool with_out) {
    const int64_t items = std::max<int64_t>(std::max(g.fwd.n_items, g.back.n_items), 1);
    const int64_t Q = kTileQ;
    const int64_t hot = (int64_t)hot_chunks(g) * g.hot.n;
    // Per (node, query): r, pi (4 + 4 B) and q (2 B) for U; carry (4 B) and zh (2 B) for V and attributes.
    return Q * (10 * g.n_u + 6 * std::max<int64_t>(g.n_v + g.n_a, 1) + 4 * (items + hot + (with_out ? g.n_u : 0))) +
           (int64_t)sizeof(TileCtl) + (int64_t)batch_cap(g) * Q * (2 * 4 + 5 * 8) + (int64_t)g.grid_cap * Q * 8 +
           (int64_t)kCtlSlices * Q * 12;
}

void ensure_batch_state(Graph &g, BatchState &b, int tiles, bool with_out) {
    if (b.tiles >= tiles && (b.out || !with_out)) return;
    free_batch_state(b);
    const int64_t items = std::max<int64_t>(std::max(g.fwd.n_items, g.back.n_items), 1);
    const size_t T = (size_t)tiles, Q = kTileQ;
    b.r = (float *)dev_alloc(g, T * g.n_u * Q * 4, "batch residues");
    b.pi = (float *)dev_alloc(g, T * g.n_u * Q * 4, "batch reserves");
    const size_t n_x = (size_t)std::max<int64_t>(g.n_v + g.n_a, 1);
    b.q = (uint16_t *)dev_alloc(g, T * g.n_u * Q * 2, "batch transport residues");
    b.c = (float *)dev_alloc(g, T * n_x * Q * 4, "batch V/attribute carries");
    b.zh = (uint16_t *)dev_alloc(g, T * n_x * Q * 2, "batch V/attribute transport residues");
    b.part = (float *)dev_alloc(g, T * items * Q * 4, "batch chunk partials");
    b.ctl = (TileCtl *)dev_alloc(g, T * sizeof(TileCtl), "batch control");
    b.blk_max = (float *)dev_alloc(g, T * 2 * batch_cap(g) * Q * 4, "batch workgroup maxima");
    b.blk_np = (unsigned long long *)dev_alloc(g, T * 5 * batch_cap(g) * Q * 8, "batch workgroup counts");
    b.red_max = (float *)dev_alloc(g, T * kCtlSlices * Q * 4, "batch control slices");
    b.red_np = (unsigned long long *)dev_alloc(g, T * kCtlSlices * Q * 8, "batch control slices");
    if (g.hot.n > 0)
        b.hot_part = (float *)dev_alloc(g, T * (size_t)hot_chunks(g) * g.hot.n * Q * 4, "batch hot-row partials");
    if (with_out) b.out = (float *)dev_alloc(g, T * Q * g.n_u * 4, "batch scores");
    b.sums = (double *)dev_alloc(g, T * g.grid_cap * Q * 8, "batch sums");
    b.tiles = tiles;
    b.grid_x = batch_cap(g);
}

namespace {
// Zeroes r, pi, q and the carries of tiles [0, nt) (zh is rewritten by every
// round's V / attribute half-step before it is read).
void clear_tiles(Graph &g, BatchState &b, int nt, hipStream_t s) {
    const int64_t tile_u = g.n_u * kTileQ, tile_x = std::max<int64_t>(g.n_v + g.n_a, 1) * kTileQ;
    hipLaunchKernelGGL(kb_fill, dim3(4096), dim3(kBlock), 0, s, b.r, (int64_t)nt * tile_u);
    hipLaunchKernelGGL(kb_fill, dim3(4096), dim3(kBlock), 0, s, b.pi, (int64_t)nt * tile_u);
    hipLaunchKernelGGL(kb_fill, dim3(4096), dim3(kBlock), 0, s, reinterpret_cast<float *>(b.q),
                       (int64_t)nt * tile_u / 2);
    hipLaunchKernelGGL(kb_fill, dim3(4096), dim3(kBlock), 0, s, b.c, (int64_t)nt * tile_x);
}
}  // namespace

void batch_init(Graph &g, BatchState &b, int nt, const int32_t *sources, const float *eps_f, int64_t n_q,
                int32_t max_iters, hipStream_t s) {
    const int64_t tile_u = g.n_u * kTileQ;
    clear_tiles(g, b, nt, s);
    std::vector<InitQuery> hq((size_t)nt * kTileQ);
    const int64_t n_valid = std::min<int64_t>(n_q, (int64_t)nt * kTileQ);
    for (int64_t i = 0; i < n_valid; ++i) hq[i] = InitQuery{g.u_new_host[(size_t)sources[i]], eps_f[i]};
    InitQuery *dq = nullptr;
    check_hip(hipMallocAsync((void **)&dq, hq.size() * sizeof(InitQuery), s), "batch init");
    check_hip(hipMemcpyAsync(dq, hq.data(), hq.size() * sizeof(InitQuery), hipMemcpyHostToDevice, s), "batch init");
    hipLaunchKernelGGL(kb_init, dim3(nt), dim3(kTileQ), 0, s, b.ctl, b.r, b.q, tile_u, dq, n_valid, max_iters);
    check_hip(hipFreeAsync(dq, s), "batch init");
    check_hip(hipGetLastError(), "batch init launch");
}

void batch_round(Graph &g, BatchState &b, int nt, hipStream_t s) {
    const BPlan p = bplan(g, nt);
    const BackSched bs = back_sched(g);
    const HotSet &hs = g.hot;
    const int64_t tile_u = g.n_u * kTileQ, tile_x = std::max<int64_t>(g.n_v + g.n_a, 1) * kTileQ;
    const int64_t tile_part = std::max<int64_t>(std::max(g.fwd.n_items, g.back.n_items), 1) * kTileQ;
    const int64_t sf = 2 * (int64_t)batch_cap(g) * kTileQ, su = 5 * (int64_t)batch_cap(g) * kTileQ;
    BArgs back{g.back.off, g.back.col, g.back.w, bs.items, bs.n_items, bs.split, bs.n_split,
               b.q, b.c, b.zh, nullptr, g.inv_b, b.part, b.ctl, tile_u, tile_x, 0, tile_part, nullptr, b.blk_np, sf,
               su, (float)g.alpha};
    // Slots of the n_p partials: 0 back, 1 back fix, 2 fwd, 3 fwd fix, 4 hot
    // rows; of the max partials: 0 fwd, 1 fwd fix; slots are batch_cap
    // workgroups apart.
    const int64_t slot = (int64_t)batch_cap(g) * kTileQ;
    // Bytes of a launch, two ways (q = running queries).  Gathered: the CSR
    // entries and offsets once, one 2-byte transport value per (entry, query),
    // and the per-(row, query) state the epilogue reads and writes.
    // Compulsory: the CSR once, the gathered transport table once per query
    // (every column once), and the same per-row state; the gap between the
    // two is what caches must absorb.  The hot-row pass reads the hot list
    // and its segment offsets once and each query's transport row of every U
    // node once, and writes and re-reads its chunk partials (both counts).
    const double q = (double)b.live_q;
    const double wb = g.fwd.w ? 8.0 : 4.0;
    const double n_x = (double)std::max<int64_t>(g.n_v + g.n_a, 1);
    const double back_csr = 8.0 * bs.nnz + 12.0 * bs.rows, back_row = 10.0 * bs.rows;  // carry r/w, zh w
    const double fwd_csr = wb * g.fwd.nnz + 8.0 * g.fwd.n_rows, fwd_row = 18.0 * g.fwd.n_rows;  // r, pi r/w, q w
    const double back_bytes = back_csr + q * (2.0 * bs.nnz + back_row);
    const double back_comp = back_csr + q * (2.0 * g.n_u + back_row);
    const double fwd_bytes = fwd_csr + q * (2.0 * g.fwd.nnz + fwd_row);
    const double fwd_comp = fwd_csr + q * (2.0 * n_x + fwd_row);
    int64_t hot_kc = 0, n_ch = 0;
    if (hs.n > 0) dense_chunking(g.n_u, &hot_kc, &n_ch);
    const double hot_bytes = 6.0 * (double)(hot_kc * n_ch) * kHotMax + 12.0 * hs.n +
                             q * (2.0 * g.n_u + 8.0 * (double)n_ch * hs.n + 10.0 * hs.n);
    if (p.back)
        profiled(g.prof, 2, back_bytes, back_comp, s, [&] {
            hipLaunchKernelGGL((kb_gather<false, kBBack>), dim3(p.back, nt), dim3(kBlock), 0, s, back,
                               (const int32_t *)g.back.col, (const float *)g.back.w);
        });
    if (p.back_fix) {
        BArgs a = back;
        a.blk_np += slot;
        hipLaunchKernelGGL((kb_fix<kBBack>), dim3(p.back_fix, nt), dim3(kBlock), 0, s, a);
    }
    if (hs.n > 0) {
        const int64_t tile_hot = n_ch * hs.n * kTileQ;
        HotReduceArgs ra{b.hot_part, tile_hot, hs.rows, hs.len, g.inv_b, b.c, b.zh, tile_x, b.blk_np + 4 * slot, su,
                         b.ctl, hs.n, (int)n_ch};
        profiled(g.prof, 4, hot_bytes, hot_bytes, s, [&] {
            launch_hot_dense(g, b.q, tile_u, b.ctl, nt, b.hot_part, tile_hot, s);
            hipLaunchKernelGGL(kb_hot_reduce, dim3((unsigned)hs.n, nt), dim3(kBlock), 0, s, ra);
        });
    }
    BArgs fwd{g.fwd.off, g.fwd.col, g.fwd.w, g.fwd.items, g.fwd.n_items, g.fwd.split, g.fwd.n_split,
              b.zh, b.r, b.q, b.pi, nullptr, b.part, b.ctl, tile_x, tile_u, tile_u, tile_part, b.blk_max,
              b.blk_np + 2 * slot, sf, su, (float)g.alpha};
    profiled(g.prof, 3, fwd_bytes, fwd_comp, s, [&] {
        if (g.unit)
            hipLaunchKernelGGL((kb_gather<true, kBFwd>), dim3(p.fwd, nt), dim3(kBlock), 0, s, fwd,
                               (const int32_t *)g.fwd.col, (const float *)nullptr);
        else
            hipLaunchKernelGGL((kb_gather<false, kBFwd>), dim3(p.fwd, nt), dim3(kBlock), 0, s, fwd,
                               (const int32_t *)g.fwd.col, (const float *)g.fwd.w);
    });
    if (p.fwd_fix) {
        BArgs a = fwd;
        a.blk_max += slot;
        a.blk_np += slot;
        hipLaunchKernelGGL((kb_fix<kBFwd>), dim3(p.fwd_fix, nt), dim3(kBlock), 0, s, a);
    }
    hipLaunchKernelGGL(kb_control_partials, dim3(kCtlSlices, nt), dim3(kCtlThreads), 0, s, b.ctl, b.blk_max,
                       b.blk_np, sf, su, batch_cap(g), (int)p.back, (int)p.back_fix, (int)p.fwd, (int)p.fwd_fix, hs.n,
                       b.red_max, b.red_np);
    hipLaunchKernelGGL(kb_control, dim3(nt), dim3(kTileQ), 0, s, b.ctl, b.red_max, b.red_np, make_rule(g));
    check_hip(hipGetLastError(), "batch round launch");
}

TuneResult batch_tune(Graph &g, int max_tiles, hipStream_t s) {
    // Sources: the first tiles * kTileQ nodes of U, at a tiny eps so no
    // query stops during the probe.  A pull-form round reads every CSR entry
    // whatever the frontier, so its cost is the same from the first round.
    const int kProbe = 3;
    TuneResult best{0, 1, 0, 0.0, 0.0};
    g.tuned_tiles = 0;
    g.tuned_wg_mult = 1;
    ++g.plan_gen;
    const bool prof = g.prof.on;
    g.prof.on = false;
    std::vector<int> tiles;
    for (int t = 1; t <= std::max(1, max_tiles); t *= 2) tiles.push_back(t);
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "tune");
    check_hip(hipEventCreate(&e1), "tune");
    double best_ms = 1e300;
    for (int nt : tiles) {
        ensure_batch_state(g, g.batch, nt, false);
        const int64_t n_q = std::min<int64_t>((int64_t)nt * kTileQ, g.n_u);
        std::vector<int32_t> src((size_t)n_q);
        std::vector<float> eps_f((size_t)n_q, 1e-30f);
        for (int64_t i = 0; i < n_q; ++i) src[i] = (int32_t)i;
        for (int mult : {1, 2, 4, 8}) {
            if (mult > 1 && std::max(64, (mult / 2) * g.grid_cap / nt) >= batch_cap(g)) break;  // same plan as before
            g.tuned_wg_mult = mult;
            batch_init(g, g.batch, nt, src.data(), eps_f.data(), n_q, 1 << 20, s);
            g.batch.live_q = n_q;
            batch_round(g, g.batch, nt, s);
            check_hip(hipEventRecord(e0, s), "tune");
            for (int i = 0; i < kProbe; ++i) batch_round(g, g.batch, nt, s);
            check_hip(hipEventRecord(e1, s), "tune");
            check_hip(hipEventSynchronize(e1), "tune");
            float ms = 0.0f;
            check_hip(hipEventElapsedTime(&ms, e0, e1), "tune");
            const double per = (double)ms / (kProbe * nt);
            ++best.candidates;
            if (nt == tiles.back() && mult == 1) best.default_ms_per_tile_round = per;
            if (per < best_ms) {
                best_ms = per;
                best.tiles = nt;
                best.wg_mult = mult;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    best.ms_per_tile_round = best_ms;
    g.tuned_tiles = best.tiles;
    g.tuned_wg_mult = best.wg_mult;
    ++g.plan_gen;
    g.prof.on = prof;
    return best;
}

void batch_rounds(Graph &g, BatchState &b, int nt, int n, hipStream_t s) {
    if (!graphs_enabled(g)) {
        for (int i = 0; i < n; ++i) batch_round(g, b, nt, s);
        return;
    }
    if (b.graphs_gen != g.plan_gen) {
        for (auto &e : b.round_graphs) (void)hipGraphExecDestroy(e.second);
        b.round_graphs.clear();
        b.graphs_gen = g.plan_gen;
    }
    hipGraphExec_t ex = nullptr;
    for (auto &e : b.round_graphs)
        if (e.first == nt) ex = e.second;
    if (!ex) {
        ex = capture_graph(g, "batch round capture", [&](hipStream_t cs) { batch_round(g, b, nt, cs); });
        b.round_graphs.emplace_back(nt, ex);
    }
    for (int i = 0; i < n; ++i) check_hip(hipGraphLaunch(ex, s), "round graph launch");
}

void batch_scores(Graph &g, BatchState &b, int nt, int64_t n_rows, float *out, hipStream_t s) {
    const int64_t tile_u = g.n_u * kTileQ;
    hipLaunchKernelGGL(kb_transpose, dim3((unsigned)((g.n_u + kWave - 1) / kWave), nt), dim3(kBlock), 0, s, b.pi,
                       tile_u, (const int32_t *)g.u_new, g.n_u, out, std::min<int64_t>(n_rows, (int64_t)nt * kTileQ));
    check_hip(hipGetLastError(), "batch scores launch");
}

void batch_resid_sums(Graph &g, BatchState &b, int t0, int nt, double *sums, hipStream_t s) {
    const int64_t tile_u = g.n_u * kTileQ;
    const unsigned gx = capped(g.n_u, kWavesPerBlock * 64, std::min(g.grid_cap, 1024));
    hipLaunchKernelGGL(kb_sums, dim3(gx, nt), dim3(kBlock), 0, s, b.r + t0 * tile_u, tile_u, g.n_u, b.sums);
    std::vector<double> h((size_t)nt * gx * kTileQ);
    check_hip(hipMemcpyAsync(h.data(), b.sums, h.size() * 8, hipMemcpyDeviceToHost, s), "batch sums D2H");
    check_hip(hipStreamSynchronize(s), "batch sums");
    for (int t = 0; t < nt; ++t)
        for (int q = 0; q < kTileQ; ++q) {
            double v = 0.0;
            for (unsigned i = 0; i < gx; ++i) v += h[((size_t)t * gx + i) * kTileQ + q];
            sums[(size_t)t * kTileQ + q] = v;
        }
}

void batch_empty(Graph &g, BatchState &b, int nt, hipStream_t s) {
    const int64_t tile_u = g.n_u * kTileQ;
    clear_tiles(g, b, nt, s);
    hipLaunchKernelGGL(kb_init, dim3(nt), dim3(kTileQ), 0, s, b.ctl, b.r, b.q, tile_u, (const InitQuery *)nullptr,
                       (int64_t)0, (int32_t)1);
    check_hip(hipGetLastError(), "batch empty launch");
}

void batch_admit(Graph &g, BatchState &b, const std::vector<AdmitReq> &reqs, int32_t max_iters, hipStream_t s) {
    if (reqs.empty()) return;
    const int64_t tile_u = g.n_u * kTileQ;
    std::vector<unsigned long long> masks((size_t)b.tiles * kMaskWords, 0ull);
    for (const AdmitReq &a : reqs) masks[(size_t)a.tile * kMaskWords + a.lane / 64] |= 1ull << (a.lane % 64);
    unsigned long long *dm = nullptr;
    AdmitReq *dr = nullptr;
    check_hip(hipMallocAsync((void **)&dm, masks.size() * 8, s), "admit");
    check_hip(hipMallocAsync((void **)&dr, reqs.size() * sizeof(AdmitReq), s), "admit");
    check_hip(hipMemcpyAsync(dm, masks.data(), masks.size() * 8, hipMemcpyHostToDevice, s), "admit");
    std::vector<AdmitReq> dev_reqs(reqs);  // sources in the device numbering
    for (AdmitReq &a : dev_reqs) a.source = g.u_new_host[(size_t)a.source];
    check_hip(hipMemcpyAsync(dr, dev_reqs.data(), dev_reqs.size() * sizeof(AdmitReq), hipMemcpyHostToDevice, s),
              "admit");
    const unsigned gx = capped(g.n_u, kWavesPerBlock * 16, 1024);
    const int64_t n_x = std::max<int64_t>(g.n_v + g.n_a, 1);
    hipLaunchKernelGGL(kb_clear_lanes, dim3(gx, b.tiles), dim3(kBlock), 0, s, b.r, b.q, b.pi, tile_u, g.n_u, b.c,
                       n_x * kTileQ, n_x, dm);
    hipLaunchKernelGGL(kb_admit, dim3(capped((int64_t)reqs.size(), kBlock, 1 << 20)), dim3(kBlock), 0, s, b.ctl, b.r,
                       b.q,
                       tile_u, dr, (int)reqs.size(), max_iters);
    check_hip(hipFreeAsync(dm, s), "admit");
    check_hip(hipFreeAsync(dr, s), "admit");
    check_hip(hipGetLastError(), "admit launch");
}

void batch_lanes_out(Graph &g, BatchState &b, int tile, const int32_t *d_lanes, int n_sel, float *out,
                     hipStream_t s) {
    if (n_sel <= 0) return;
    const int64_t tile_u = g.n_u * kTileQ;
    hipLaunchKernelGGL(kb_gather_lanes, dim3((unsigned)((g.n_u + kWave - 1) / kWave)), dim3(kBlock), 0, s,
                       b.pi + tile * tile_u, (const int32_t *)g.u_new, g.n_u, d_lanes, n_sel, out);
    check_hip(hipGetLastError(), "lanes out launch");
}

}  // namespace ahpp
