// Small device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ahpp {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Orders the wave's earlier LDS writes before its later LDS reads (other lanes).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix sum over the 256 threads of a workgroup.  `lds` must hold
// 4 elements; *total receives the workgroup sum.  Contains __syncthreads.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *lds, T *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T t = lds[i];
        if (i < wid) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Sum over the 256 threads of a workgroup (result valid in every thread).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
    T tot;
    (void)block_exclusive_scan<T>(v, lds, &tot);
    return tot;
}

__device__ __forceinline__ float block_max_f(float v, float *lds) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    float m = fmaxf(fmaxf(lds[0], lds[1]), fmaxf(lds[2], lds[3]));
    __syncthreads();
    return m;
}

// Max and sum over a workgroup of kWaves waves; lds holds kWaves entries.
template <int kWaves>
__device__ __forceinline__ float block_max_n(float v, float *lds) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = lds[0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) m = fmaxf(m, lds[i]);
    __syncthreads();
    return m;
}

template <int kWaves>
__device__ __forceinline__ unsigned long long block_sum_u64_n(unsigned long long v, unsigned long long *lds) {
    v = wave_sum_u64(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long m = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) m += lds[i];
    __syncthreads();
    return m;
}

}  // namespace ahpp
