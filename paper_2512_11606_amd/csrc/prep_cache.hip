// Key of a graph's inputs and the cache of its Theorem 3 lambda.
//
// The key is 128 bits: for each of two lanes, the sum (mod 2^64) over every
// element of every input array of a SplitMix64-mixed word of (lane, array,
// position, value), folded with the sizes, alpha, beta and the Theorem 3
// round count.  A sum of per-element mixes has no order of its own, so the
// device (at load, on the uploaded arrays) and the host (ahpp_graph_key)
// reach the same value.  Any changed id, weight or parameter changes it.
//
// The cache holds, per key, lambda of Eq. 6: the part of a load worth
// keeping.  Its T sweeps of the whole graph cost more than the device build
// of the CSRs from the COO, whose time is mostly the upload of the COO
// itself; a file of the built CSRs would be larger than the COO (every
// entry twice, plus schedules) and slower to read back than to rebuild.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ahpp_internal.h"

namespace ahpp {

namespace {

constexpr uint64_t kLane[2] = {0x9E3779B97F4A7C15ull, 0xC2B2AE3D27D4EB4Full};

// The SplitMix64 finaliser (Steele, Lea and Flood, 2014).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The word element `pos` of array `arr` with 32-bit pattern `v` adds to lane l.
__host__ __device__ inline uint64_t elem_word(int l, uint32_t arr, uint64_t pos, uint32_t v) {
    return mix64(mix64(kLane[l] + pos * 8u + arr) + v);
}

__global__ void k_key_sum(const uint32_t *__restrict__ v, int64_t n, uint32_t arr, unsigned long long *sums) {
    __shared__ unsigned long long s0[kBlock], s1[kBlock];
    unsigned long long a = 0, b = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a += elem_word(0, arr, (uint64_t)i, v[i]);
        b += elem_word(1, arr, (uint64_t)i, v[i]);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s0[threadIdx.x] += s0[threadIdx.x + o];
            s1[threadIdx.x] += s1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&sums[0], s0[0]);
        atomicAdd(&sums[1], s1[0]);
    }
}

// The sizes and parameters folded into both lanes.
void finish_key(const KeyInput &in, const uint64_t sums[2], uint64_t key[2]) {
    uint64_t a, b;
    std::memcpy(&a, &in.alpha, 8);
    std::memcpy(&b, &in.beta, 8);
    const uint64_t p[] = {(uint64_t)in.n_u, (uint64_t)in.n_v, (uint64_t)in.n_attr, (uint64_t)in.n_edges,
                          (uint64_t)in.n_assoc, (uint64_t)(in.has_ew ? 1 : 0) | (uint64_t)(in.has_aw ? 2 : 0),
                          a, b, (uint64_t)(int64_t)in.lambda_iters, 1u /* key format */};
    for (int l = 0; l < 2; ++l) {
        uint64_t h = kLane[l];
        for (uint64_t x : p) h = mix64(h ^ x);
        key[l] = mix64(h ^ sums[l]);
    }
}

}  // namespace

void coo_key_device(const KeyInput &in, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                    const int32_t *aa, const float *aw, uint64_t key[2], hipStream_t s) {
    DevTemp<unsigned long long> sums_(2, "graph key");
    unsigned long long *d = sums_.get();
    check_hip(hipMemsetAsync(d, 0, 16, s), "graph key");
    const void *arrs[6] = {eu, ev, ew, au, aa, aw};
    const int64_t lens[6] = {in.n_edges, in.n_edges, in.n_edges, in.n_assoc, in.n_assoc, in.n_assoc};
    for (uint32_t k = 0; k < 6; ++k) {
        if (!arrs[k] || lens[k] <= 0) continue;
        const int64_t blocks = std::min<int64_t>((lens[k] + kBlock - 1) / kBlock, 8192);
        hipLaunchKernelGGL(k_key_sum, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const uint32_t *)arrs[k], lens[k], k,
                           d);
    }
    check_hip(hipGetLastError(), "graph key launch");
    unsigned long long h[2];
    check_hip(hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, s), "graph key D2H");
    check_hip(hipStreamSynchronize(s), "graph key");
    const uint64_t sums[2] = {h[0], h[1]};
    finish_key(in, sums, key);
}

void coo_key_host(const KeyInput &in, const int32_t *eu, const int32_t *ev, const float *ew, const int32_t *au,
                  const int32_t *aa, const float *aw, uint64_t key[2]) {
    const uint32_t *arrs[6] = {(const uint32_t *)eu, (const uint32_t *)ev, (const uint32_t *)ew,
                               (const uint32_t *)au, (const uint32_t *)aa, (const uint32_t *)aw};
    const int64_t lens[6] = {in.n_edges, in.n_edges, in.n_edges, in.n_assoc, in.n_assoc, in.n_assoc};
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<uint64_t> part((size_t)nth * 2, 0);
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t) {
        pool.emplace_back([&, t] {
            uint64_t a = 0, b = 0;
            for (uint32_t k = 0; k < 6; ++k) {
                if (!arrs[k] || lens[k] <= 0) continue;
                const int64_t lo = lens[k] * t / nth, hi = lens[k] * (t + 1) / nth;
                for (int64_t i = lo; i < hi; ++i) {
                    a += elem_word(0, k, (uint64_t)i, arrs[k][i]);
                    b += elem_word(1, k, (uint64_t)i, arrs[k][i]);
                }
            }
            part[(size_t)t * 2] = a;
            part[(size_t)t * 2 + 1] = b;
        });
    }
    for (auto &th : pool) th.join();
    uint64_t sums[2] = {0, 0};
    for (int t = 0; t < nth; ++t) {
        sums[0] += part[(size_t)t * 2];
        sums[1] += part[(size_t)t * 2 + 1];
    }
    finish_key(in, sums, key);
}

namespace {
constexpr char kMagic[8] = {'A', 'H', 'P', 'P', 'L', 'A', 'M', '1'};

struct LambdaRecord {
    char magic[8];
    uint64_t key[2];
    int64_t n_u, n_v, n_attr, n_edges, n_assoc;
    double alpha, beta;
    int32_t lambda_iters, pad;
    double lambda;
};

std::string cache_path(const std::string &dir, const uint64_t key[2]) {
    char name[64];
    std::snprintf(name, sizeof(name), "ahpp-%016" PRIx64 "%016" PRIx64 ".lambda", key[0], key[1]);
    return dir + "/" + name;
}

bool matches(const LambdaRecord &r, const KeyInput &in, const uint64_t key[2]) {
    return std::memcmp(r.magic, kMagic, 8) == 0 && r.key[0] == key[0] && r.key[1] == key[1] && r.n_u == in.n_u &&
           r.n_v == in.n_v && r.n_attr == in.n_attr && r.n_edges == in.n_edges && r.n_assoc == in.n_assoc &&
           r.alpha == in.alpha && r.beta == in.beta && r.lambda_iters == in.lambda_iters && r.lambda > 0.0;
}
}  // namespace

bool lambda_cache_read(const std::string &dir, const KeyInput &in, const uint64_t key[2], double *lambda) {
    FILE *f = std::fopen(cache_path(dir, key).c_str(), "rb");
    if (!f) return false;
    LambdaRecord r;
    const bool ok = std::fread(&r, sizeof(r), 1, f) == 1 && matches(r, in, key);
    std::fclose(f);
    if (ok) *lambda = r.lambda;
    return ok;
}

bool lambda_cache_write(const std::string &dir, const KeyInput &in, const uint64_t key[2], double lambda) {
    LambdaRecord r;
    std::memset(&r, 0, sizeof(r));
    std::memcpy(r.magic, kMagic, 8);
    r.key[0] = key[0];
    r.key[1] = key[1];
    r.n_u = in.n_u;
    r.n_v = in.n_v;
    r.n_attr = in.n_attr;
    r.n_edges = in.n_edges;
    r.n_assoc = in.n_assoc;
    r.alpha = in.alpha;
    r.beta = in.beta;
    r.lambda_iters = in.lambda_iters;
    r.lambda = lambda;
    const std::string path = cache_path(dir, key);
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>{}(
                                                 std::this_thread::get_id()));
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool wrote = std::fwrite(&r, sizeof(r), 1, f) == 1;
    const bool closed = std::fclose(f) == 0;
    if (!wrote || !closed || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace ahpp
