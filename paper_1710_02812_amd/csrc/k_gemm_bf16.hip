// Passes over A on the matrix cores, for mixed-precision plans:
//   op 0: Y = A_blk * X,   op 1: Y = A_blk^T * X,
// with A (float32, row-major) and X (float64 col-major panel; rounded to float32
// first) rounded to bfloat16 (nearest even), products summed in float32 by
// v_mfma_f32_16x16x32_bf16, and Y written as float64.
//
// A 256-thread work-group owns a 128 x 64 output tile; wave w computes rows
// [32w, 32w + 32) as 2 x 4 MFMA tiles of 16 x 16.  The reduction streams in slabs
// of 32: each slab of A and X is read from global memory (coalesced along the
// contiguous dimension; the transpose of op 1 happens on the way into LDS),
// converted, and stored k-contiguous in LDS so that each lane's MFMA operand is
// one aligned 16-byte read.  The next slab is loaded into registers while the
// matrix cores work on the current one.
//
// MFMA 16x16x32 operand layout (lane l of 64): A fragment row l % 16, reduction
// indices 8 (l / 16) .. 8 (l / 16) + 7; B fragment column l % 16, same reduction
// indices; the 4 accumulators of lane l hold column l % 16, rows 4 (l / 16) + i.
#include "hsvd_internal.hpp"

namespace hsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 64, BK = 32;
constexpr int PITCH = BK + 8;   // bf16 per LDS row: 80 bytes, keeps 16-byte alignment

template <int OP>
__global__ __launch_bounds__(256) void k_gemm_bf16(const void* const* __restrict__ ptrs,
                                                   double* __restrict__ ws,
                                                   const GemmTask* __restrict__ tasks,
                                                   const TileRef* __restrict__ tiles, int N) {
    __shared__ __attribute__((aligned(16))) __bf16 As[BM * PITCH];   // [out row][k]
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN * PITCH];   // [out col][k]
    const TileRef tr = tiles[blockIdx.x];
    const GemmTask t = tasks[tr.task];
    const int nct = (N + BN - 1) / BN;
    const int r0 = (tr.tile / nct) * BM, c0 = (tr.tile % nct) * BN;
    const int out_rows = OP == 0 ? t.rows : t.cols;
    const int K = OP == 0 ? t.cols : t.rows;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float* Ab = (const float*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;

    float ra[16];
    float rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int r, kk;
            if (OP == 0) { r = (tid >> 5) + 8 * u; kk = tid & 31; }
            else { r = tid & 127; kk = (tid >> 7) + 2 * u; }
            const int gr = r0 + r, gk = k0 + kk;
            float v = 0.0f;
            if (gr < out_rows && gk < K)
                v = OP == 0 ? Ab[(int64_t)gr * lda + gk] : Ab[(int64_t)gk * lda + gr];
            ra[u] = v;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = (tid >> 5) + 8 * u, kk = tid & 31;
            const int gc = c0 + c, gk = k0 + kk;
            rb[u] = (gc < N && gk < K) ? (float)X[(int64_t)gc * t.x_ld + gk] : 0.0f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int r, kk;
            if (OP == 0) { r = (tid >> 5) + 8 * u; kk = tid & 31; }
            else { r = tid & 127; kk = (tid >> 7) + 2 * u; }
            As[r * PITCH + kk] = (__bf16)ra[u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = (tid >> 5) + 8 * u, kk = tid & 31;
            Bs[c * PITCH + kk] = (__bf16)rb[u];
        }
    };

    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const int fr = lane & 15, fk = 8 * (lane >> 4);
    load(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        stash();
        __syncthreads();
        if (k0 + BK < K) load(k0 + BK);
        bf16x8 a[2], b[4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *(const bf16x8*)&As[(32 * wave + 16 * i + fr) * PITCH + fk];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8*)&Bs[(16 * j + fr) * PITCH + fk];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int gc = c0 + 16 * j + fr;
        if (gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gr = r0 + 32 * wave + 16 * i + 4 * (lane >> 4) + e;
                if (gr < out_rows) Y[(int64_t)gc * t.y_ld + gr] = (double)acc[i][j][e];
            }
    }
}

hipError_t launch_gemm_bf16(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                            const TileRef* tiles, int ntiles, int N, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 g(ntiles), b(256);
    if (op == 0)
        hipLaunchKernelGGL(k_gemm_bf16<0>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
    else
        hipLaunchKernelGGL(k_gemm_bf16<1>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
    return hipGetLastError();
}

}  // namespace hsvd
