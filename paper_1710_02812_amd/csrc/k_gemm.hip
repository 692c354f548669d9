// Products of blocks of the input A with thin panels (the passes over A):
//   op 0: Y = A_blk * X      (leaf sketch / power step / projection Y = A V)
//   op 1: Y = A_blk^T * X    (leaf power step / slab re-projection W^T = A_i^T U_i)
// A is row-major (float64 or float32), taken from the plan's pointer table by the
// task's matrix index; X and Y are float64 col-major panels.
// One 256-thread work-group computes a 64 x 64 output tile; the reduction
// dimension streams through LDS in slabs of 32 with coalesced row reads of A.
#include "hsvd_internal.hpp"

namespace hsvd {

constexpr int GT = 64;   // output tile (rows and columns)
constexpr int GK = 32;   // reduction slab

template <typename TA>
__global__ __launch_bounds__(256) void k_gemm_ax(const void* const* __restrict__ ptrs,
                                                 double* __restrict__ ws,
                                                 const GemmTask* __restrict__ tasks,
                                                 const TileRef* __restrict__ tiles, int N) {
    __shared__ double As[GK][GT + 1];   // [k][row]
    __shared__ double Xs[GK][GT + 1];   // [k][col]
    const TileRef tr = tiles[blockIdx.x];
    const GemmTask t = tasks[tr.task];
    const int nct = (N + GT - 1) / GT;
    const int r0 = (tr.tile / nct) * GT, c0 = (tr.tile % nct) * GT;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const TA* Ab = (const TA*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int k0 = 0; k0 < t.cols; k0 += GK) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int r = e >> 5, kk = e & 31;
            const int gr = r0 + r, gk = k0 + kk;
            As[kk][r] = (gr < t.rows && gk < t.cols) ? (double)Ab[(int64_t)gr * lda + gk] : 0.0;
            const int c = e >> 5;
            const int gc = c0 + c;
            Xs[kk][c] = (gc < N && gk < t.cols) ? X[(int64_t)gc * t.x_ld + gk] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < GK; ++kk) {
            double a[4], x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = Xs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], x[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int gc = c0 + tx + 16 * j;
        if (gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gr = r0 + ty + 16 * i;
            if (gr < t.rows) Y[(int64_t)gc * t.y_ld + gr] = acc[i][j];
        }
    }
}

template <typename TA>
__global__ __launch_bounds__(256) void k_gemm_atx(const void* const* __restrict__ ptrs,
                                                  double* __restrict__ ws,
                                                  const GemmTask* __restrict__ tasks,
                                                  const TileRef* __restrict__ tiles, int N) {
    __shared__ double As[GK][GT + 1];   // [k = A row][A column]
    __shared__ double Xs[GK][GT + 1];   // [k][col]
    const TileRef tr = tiles[blockIdx.x];
    const GemmTask t = tasks[tr.task];
    const int nct = (N + GT - 1) / GT;
    const int r0 = (tr.tile / nct) * GT, c0 = (tr.tile % nct) * GT;  // r0: A column
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const TA* Ab = (const TA*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int k0 = 0; k0 < t.rows; k0 += GK) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int kk = e >> 6, c = e & 63;
            const int gk = k0 + kk, gc = r0 + c;
            As[kk][c] = (gk < t.rows && gc < t.cols) ? (double)Ab[(int64_t)gk * lda + gc] : 0.0;
            const int xc = e >> 5, xk = e & 31;
            const int gxc = c0 + xc, gxk = k0 + xk;
            Xs[xk][xc] = (gxc < N && gxk < t.rows) ? X[(int64_t)gxc * t.x_ld + gxk] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < GK; ++kk) {
            double a[4], x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = Xs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], x[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int gc = c0 + tx + 16 * j;
        if (gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int gr = r0 + ty + 16 * i;
            if (gr < t.cols) Y[(int64_t)gc * t.y_ld + gr] = acc[i][j];
        }
    }
}

hipError_t launch_gemm(int op, int fp32, const void* const* ptrs, double* ws,
                       const GemmTask* tasks, const TileRef* tiles, int ntiles, int N,
                       hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 g(ntiles), b(256);
    if (op == 0) {
        if (fp32)
            hipLaunchKernelGGL(k_gemm_ax<float>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
        else
            hipLaunchKernelGGL(k_gemm_ax<double>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
    } else {
        if (fp32)
            hipLaunchKernelGGL(k_gemm_atx<float>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
        else
            hipLaunchKernelGGL(k_gemm_atx<double>, g, b, 0, s, ptrs, ws, tasks, tiles, N);
    }
    return hipGetLastError();
}

}  // namespace hsvd
