// Peak probes of the device (measurement only, no part of the method): the rates a
// plain kernel reaches on this GPU, against which the method's kernels are read.
//   read : every thread streams 16-byte vectors, 8 loads in flight (HBM read rate);
//   copy : 16-byte loads and stores, 4 in flight (read + write rate);
//   mfma : every wave runs 4 independent accumulation chains of one matrix-core
//          instruction (float64 16x16x4, bfloat16 16x16x32 with float32 sums, float32
//          16x16x4) for `iters` steps; the grid puts 8 waves on every SIMD.
// Results are kept alive by a store that a data-dependent test never takes.
#include "hsvd_internal.hpp"

namespace hsvd {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int PT = 256;                 // threads per work-group
constexpr int PB = 2048;                // work-groups (8 per CU, 8 waves per SIMD)
constexpr float kNever = 1.2345e38f;    // a sum the probes never reach

__global__ __launch_bounds__(PT) void k_probe_read(const f32x4* __restrict__ p, int64_t n,
                                                   float* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * PT;
    int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (; i + 7 * stride < n; i += 8 * stride) {
        f32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[i + u * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; i < n; i += stride) acc += p[i];
    const float s = acc[0] + acc[1] + acc[2] + acc[3];
    if (s == kNever) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(PT) void k_probe_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                   int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * PT;
    int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        f32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

template <int KIND>
__global__ __launch_bounds__(PT) void k_probe_mfma(int iters, float* __restrict__ sink) {
    const int lane = threadIdx.x & 63;
    float s = 0.0f;
    if constexpr (KIND == 0) {
        const double a = 1e-3 * (1 + (lane & 3)), b = 1e-3;
        v4d acc[4] = {};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) s += (float)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
    } else if constexpr (KIND == 1) {
        bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(1e-3f * (1 + ((lane + e) & 3)));
            b[e] = (__bf16)1e-3f;
        }
        f32x4 acc[4] = {};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else {
        const float a = 1e-3f * (1 + (lane & 3)), b = 1e-3f;
        f32x4 acc[4] = {};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    }
    if (s == kNever) sink[blockIdx.x] = s;
}

}  // namespace

// kind 0 read, 1 copy (first half of buf to the second), 2 / 3 / 4 float64 / bfloat16 /
// float32 matrix cores; *work receives the bytes moved or the flops.
hipError_t launch_probe(int kind, void* buf, int64_t bytes, int iters, float* sink, double* work,
                        hipStream_t s) {
    if (kind == 0 || kind == 1) {
        const int64_t n = bytes / 16 / (kind == 1 ? 2 : 1);
        if (n < 1 || ((uintptr_t)buf & 15)) return hipErrorInvalidValue;
        if (kind == 0) {
            hipLaunchKernelGGL(k_probe_read, dim3(PB), dim3(PT), 0, s, (const f32x4*)buf, n, sink);
            *work = 16.0 * (double)n;
        } else {
            const f32x4* src = (const f32x4*)buf;
            hipLaunchKernelGGL(k_probe_copy, dim3(PB), dim3(PT), 0, s, src, (f32x4*)buf + n, n);
            *work = 32.0 * (double)n;
        }
        return hipGetLastError();
    }
    if (kind < 2 || kind > 4 || iters < 1) return hipErrorInvalidValue;
    // per instruction: 16 x 16 x 4 (x 2 flops) for float64 and float32, 16 x 16 x 32 for bfloat16
    const double per = kind == 3 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
    const double waves = (double)PB * (PT / 64);
    *work = waves * 4.0 * (double)iters * per;
    if (kind == 2) hipLaunchKernelGGL(k_probe_mfma<0>, dim3(PB), dim3(PT), 0, s, iters, sink);
    else if (kind == 3) hipLaunchKernelGGL(k_probe_mfma<1>, dim3(PB), dim3(PT), 0, s, iters, sink);
    else hipLaunchKernelGGL(k_probe_mfma<2>, dim3(PB), dim3(PT), 0, s, iters, sink);
    return hipGetLastError();
}

}  // namespace hsvd
