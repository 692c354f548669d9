// Products of blocks of the input A with thin panels (the passes over A):
//   op 0: Y = A_blk * X      (leaf sketch / power step / projection Y = A V)
//   op 1: Y = A_blk^T * X    (leaf power step / slab re-projection W^T = A_i^T U_i)
// A is row-major (float64 or float32), taken from the plan's pointer table by the
// task's matrix index; X and Y are float64 col-major panels.
// One 256-thread work-group computes a 64 x 64 output tile on the float64 matrix
// cores; the reduction dimension streams through LDS in slabs of 32 with
// coalesced reads of A and X.
#include "hsvd_internal.hpp"

namespace hsvd {

constexpr int GT = 64;   // output tile (rows and columns)
constexpr int GK = 32;   // reduction slab

typedef double v4d __attribute__((ext_vector_type(4)));

// One 64 x 64 output tile per 256-thread work-group on the float64 matrix cores
// (v_mfma_f64_16x16x4_f64): wave w owns the 32 x 32 quarter (rows 32 (w & 1),
// columns 32 (w >> 1)) as 2 x 2 blocks of 16 x 16.  Operands per 4-deep step:
// lane l holds A[i = l % 16][k = l / 16] and X[k = l / 16][j = l % 16]; the
// accumulator holds D[i = l / 16 + 4 v][j = l % 16] in element v.
// Slabs of 32 along the reduction are staged through LDS in the order they are
// read from memory (conflict-free stores) and the next slab is fetched into
// registers while the current one is multiplied.
//   OP 0: A slab As[row][k] (pitch 33), OP 1: As[k][A column] (pitch 65);
//   X slab Xs[col][k] (pitch 33) in both.
template <typename TA, int OP>
__global__ __launch_bounds__(256) void k_gemm_mfma(const void* const* __restrict__ ptrs,
                                                   double* __restrict__ ws,
                                                   const GemmTask* __restrict__ tasks,
                                                   const TileRef* __restrict__ tiles, int N) {
    constexpr int AP = OP == 0 ? GK + 1 : GT + 1;
    constexpr int XP = GK + 1;
    __shared__ double As[OP == 0 ? GT * AP : GK * AP];
    __shared__ double Xs[GT * XP];
    const TileRef tr = tiles[blockIdx.x];
    const GemmTask t = tasks[tr.task];
    const int nct = (N + GT - 1) / GT;
    const int r0 = (tr.tile / nct) * GT, c0 = (tr.tile % nct) * GT;
    const int M = OP == 0 ? t.rows : t.cols;      // output rows
    const int K = OP == 0 ? t.cols : t.rows;      // reduction length
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const TA* Ab = (const TA*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;

    TA pa[8];
    double px[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            if (OP == 0) {
                const int r = e >> 5, kk = e & 31;            // A[r0 + r][k0 + kk]
                const int gr = r0 + r, gk = k0 + kk;
                pa[u] = (gr < M && gk < K) ? Ab[(int64_t)gr * lda + gk] : (TA)0;
            } else {
                const int kk = e >> 6, c = e & 63;            // A[k0 + kk][r0 + c]
                const int gk = k0 + kk, gc = r0 + c;
                pa[u] = (gk < K && gc < M) ? Ab[(int64_t)gk * lda + gc] : (TA)0;
            }
            const int xc = e >> 5, xk = e & 31;                // X[k0 + xk][c0 + xc]
            const int gxc = c0 + xc, gxk = k0 + xk;
            px[u] = (gxc < N && gxk < K) ? X[(int64_t)gxc * t.x_ld + gxk] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            if (OP == 0) As[(e >> 5) * AP + (e & 31)] = (double)pa[u];
            else As[(e >> 6) * AP + (e & 63)] = (double)pa[u];
            Xs[(e >> 5) * XP + (e & 31)] = px[u];
        }
    };

    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    fetch(0);
    for (int k0 = 0; k0 < K; k0 += GK) {
        stage();
        __syncthreads();
        if (k0 + GK < K) fetch(k0 + GK);                     // in flight during the products
#pragma unroll
        for (int q = 0; q < GK / 4; ++q) {
            const int kk = 4 * q + lk;
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wr + 16 * i + li;
                a[i] = OP == 0 ? As[row * AP + kk] : As[kk * AP + row];
                b[i] = Xs[(wc + 16 * i + li) * XP + kk];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int gc = c0 + wc + 16 * j + li;
        if (gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = r0 + wr + 16 * i + lk + 4 * v;
                if (gr < M) Y[(int64_t)gc * t.y_ld + gr] = acc[i][j][v];
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
            hipLaunchKernelGGL((k_gemm_mfma<float, 0>), g, b, 0, s, ptrs, ws, tasks, tiles, N);
        else
            hipLaunchKernelGGL((k_gemm_mfma<double, 0>), g, b, 0, s, ptrs, ws, tasks, tiles, N);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_gemm_mfma<float, 1>), g, b, 0, s, ptrs, ws, tasks, tiles, N);
        else
            hipLaunchKernelGGL((k_gemm_mfma<double, 1>), g, b, 0, s, ptrs, ws, tasks, tiles, N);
    }
    return hipGetLastError();
}

}  // namespace hsvd
