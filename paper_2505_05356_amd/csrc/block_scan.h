// Wave64 / workgroup prefix sums used by the sort and emission kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace gft {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_reduce_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Exclusive scan over a workgroup of NT threads (NT multiple of 64, <= 1024).
// `scratch` must hold NT/64 + 1 elements of T.  Returns the exclusive prefix
// of the calling thread; *total receives the workgroup sum.  Contains
// barriers: every thread of the workgroup must call it.
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive_scan(T x, T* scratch, T* total) {
    constexpr int NW = NT / 64;
    const int lane = lane_id();
    const int wave = threadIdx.x / 64;
    T inc = wave_inclusive_scan(x);
    if (lane == 63) scratch[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            T v = scratch[w];
            scratch[w] = run;
            run += v;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    T res = scratch[wave] + inc - x;
    *total = scratch[NW];
    __syncthreads();
    return res;
}

}  // namespace gft
