// Device helpers shared by the gfx950 kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace hsvd {

// Arrival at a node of a reduction tree that spans work-groups (the last of `n`
// children to arrive continues with the node).  Every wave first waits for its own
// global stores; one thread then publishes them all with an agent-scope release on
// the arrival count (one L2 write-back for the block), and only the last arrival takes
// the agent-scope acquire (one L2 invalidate) before the block reads its siblings'
// results.  Fences in every wave would write back and invalidate the L2 once per wave,
// discarding the cached data of every other work-group on the same XCD.  The last
// arrival resets the count; s_flag is a __shared__ int; all threads must call it.
__device__ __forceinline__ bool tree_arrive(int* count, int n, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0x0F70);           // vmcnt(0): this wave's stores are done
    __syncthreads();
    if (threadIdx.x == 0) {
        const int old = __hip_atomic_fetch_add(count, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int last = old == n - 1;
        if (last) {
            atomicExch(count, 0);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        *s_flag = last;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Move a double between lanes with a DPP control (GFX9 encodings):
//   0xB1 quad_perm[1,0,3,2] (lane ^ 1), 0x4E quad_perm[2,3,0,1] (lane ^ 2),
//   0x141 row_half_mirror (lane i <-> 7-i within 8), 0x140 row_mirror (i <-> 15-i).
// Every control used here reads a lane of the same row, so no lane keeps an old value
// (the plain move needs no initialised destination).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// All-lane sums inside aligned groups of 2, 4, 8, 16 lanes (DPP, no LDS traffic);
// 32 and 64 add one or two cross-row exchanges.
__device__ __forceinline__ double sum2(double v) { return v + dpp_d<0xB1>(v); }
__device__ __forceinline__ double sum4(double v) { v = sum2(v); return v + dpp_d<0x4E>(v); }
__device__ __forceinline__ double sum8(double v) { v = sum4(v); return v + dpp_d<0x141>(v); }
__device__ __forceinline__ double sum16(double v) { v = sum8(v); return v + dpp_d<0x140>(v); }
__device__ __forceinline__ double sum32(double v) { v = sum16(v); return v + __shfl_xor(v, 16, 64); }
__device__ __forceinline__ double wave_sum(double v) { v = sum32(v); return v + __shfl_xor(v, 32, 64); }

// Sum over `width` consecutive aligned lanes (width a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int width) {
    switch (width) {
        case 1: return v;
        case 2: return sum2(v);
        case 4: return sum4(v);
        case 8: return sum8(v);
        case 16: return sum16(v);
        case 32: return sum32(v);
        default: return wave_sum(v);
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
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

// Reciprocal square root and reciprocal from the hardware estimates (v_rsq_f64,
// v_rcp_f64) refined by two Newton steps each, y <- y (3 - x y^2) / 2 and
// y <- y (2 - x y); each step squares the relative error.  For normal positive x.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * fma(-x, y, 2.0);
    y = y * fma(-x, y, 2.0);
    return y;
}
// sqrt(x) for x >= 0: x * rsqrt(x) plus one correction step.
__device__ __forceinline__ double sqrt_nr(double x) {
    if (x == 0.0) return 0.0;
    const double r = rsqrt_nr(x);
    const double s = x * r;
    return fma(0.5 * r, fma(-s, s, x), s);
}

}  // namespace hsvd
