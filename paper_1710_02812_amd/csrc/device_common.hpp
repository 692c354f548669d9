// Device helpers shared by the gfx950 kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace hsvd {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over `width` consecutive lanes (width a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum; `red` needs blockDim.x / 64 doubles of LDS.  Result broadcast.
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

}  // namespace hsvd
