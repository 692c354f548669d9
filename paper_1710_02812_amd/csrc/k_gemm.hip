// Products of blocks of the input A with thin panels (the passes over A):
//   op 0: Y = A_blk * X      (leaf sketch / power step / projection Y = A V)
//   op 1: Y = A_blk^T * X    (leaf power step / slab re-projection W^T = A_i^T U_i)
// A is row-major (float64 or float32), taken from the plan's pointer table by the
// task's matrix index; X and Y are float64 col-major panels.
// One 256-thread work-group computes a 64 x 64 output tile on the float64 matrix
// cores; the reduction dimension streams through LDS in slabs of 32 with
// coalesced reads of A and X.
// op 0 with an energy buffer also sums the squares of the A elements it reads: tile i
// of the launch writes its part of its block's energy ||A_blk||_F^2 (the squares of its
// 64 rows; 0 from column tiles past the first, which read the same rows) to
// ws[e_part + i], so a block's sketch and its energy take one pass over A.
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

constexpr int GT = MF_T;  // output tile (rows and columns)

// One 64 x NC output tile per 256-thread work-group on the float64 matrix cores (NC = 64,
// or 96 with 32-deep slabs when the product has 65..96 columns, so that A is read once).
//   OP 0: Y = A_blk X   (A_blk row-major: the tile's A operand as stored)
//   OP 1: Y = A_blk^T X (the stored rows of A_blk are the reduction index)
template <typename TA, int OP, int NC = MF_T, int KS = MF_K>
__global__ __launch_bounds__(256) void k_gemm_mfma(const void* const* __restrict__ ptrs,
                                                   double* __restrict__ ws,
                                                   const GemmTask* __restrict__ tasks,
                                                   const TileRef* __restrict__ tiles, int N,
                                                   const int* __restrict__ guard, int64_t e_part) {
    if (guard && *guard) return;                  // a skipped stage (every group returns)
    __shared__ double As[mfma_lds_a<OP, KS>()];
    __shared__ double Bs[mfma_lds_b<KS, NC>()];
    __shared__ double s_sq[4];
    const TileRef tr = tiles[blockIdx.x];
    const GemmTask t = tasks[tr.task];
    const int nct = gemm_f64_col_tiles(N);
    const int r0 = (tr.tile / nct) * GT, c0 = (tr.tile % nct) * NC;
    const int M = OP == 0 ? t.rows : t.cols;      // output rows
    const int K = OP == 0 ? t.cols : t.rows;      // reduction length
    const TA* Ab = (const TA*)ptrs[4 * t.mat] + t.a_off;
    v4d acc[2][NC / 32];
    double ssq = 0.0;
    mfma_tile<TA, OP, true, double, false, OP == 0, KS, NC>(Ab, t.lda, ws + t.x_off, t.x_ld, M, N, K, r0, c0, As, Bs,
                                                            acc, &ssq);
    double* Y = ws + t.y_off;
    mfma_tile_out(M, N, r0, c0, acc, [&](int r, int c, double v) { Y[(int64_t)c * t.y_ld + r] = v; });
    if (OP == 0 && e_part >= 0) {
        ssq = wave_sum(ssq);
        if ((threadIdx.x & 63) == 0) s_sq[threadIdx.x >> 6] = ssq;
        __syncthreads();
        if (threadIdx.x == 0) ws[e_part + blockIdx.x] = c0 == 0 ? (s_sq[0] + s_sq[1]) + (s_sq[2] + s_sq[3]) : 0.0;
    }
}

// Gram matrix of the input, G = X^T X (X row-major m x n, G n x n), for the plans that
// decompose X^T X: tile (ti, tj) with ti <= tj of G over the rows of chunk kc, written
// to partial kc (col-major, ld n) at (ti, tj) and mirrored at (tj, ti); the partials are
// summed by the thin-sum kernel.  refs: one GramRef per (tile, chunk).
template <typename TA>
__global__ __launch_bounds__(256) void k_gram_xtx(const void* const* __restrict__ ptrs, int mat, int64_t m,
                                                  int64_t n, int64_t rows_per_chunk, double* __restrict__ ws,
                                                  int64_t parts_off, const GramRef* __restrict__ refs) {
    __shared__ double As[mfma_lds_a<1>()];
    __shared__ double Bs[mfma_lds_b()];
    const GramRef g = refs[blockIdx.x];
    const TA* X = (const TA*)ptrs[4 * mat];
    const int64_t row0 = (int64_t)g.chunk * rows_per_chunk;
    const int K = (int)std::min<int64_t>(rows_per_chunk, m - row0);
    const int r0 = g.ti * GT, c0 = g.tj * GT;
    v4d acc[2][2];
    mfma_tile<TA, 1, true, TA, true>(X + row0 * n, n, X + row0 * n, n, (int)n, (int)n, K, r0, c0, As, Bs, acc);
    double* part = ws + parts_off + (int64_t)g.chunk * n * n;
    const bool diag = g.ti == g.tj;               // a diagonal tile writes each pair once
    mfma_tile_out((int)n, (int)n, r0, c0, acc, [&](int r, int c, double v) {
        if (diag && r > c) return;
        part[(int64_t)c * n + r] = v;
        part[(int64_t)r * n + c] = v;
    });
}

hipError_t launch_gram_xtx(int fp32, const void* const* ptrs, int mat, int64_t m, int64_t n,
                           int64_t rows_per_chunk, double* ws, int64_t parts_off, const GramRef* refs, int nrefs,
                           hipStream_t s) {
    if (nrefs <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_gram_xtx<float>, dim3(nrefs), dim3(256), 0, s, ptrs, mat, m, n, rows_per_chunk, ws,
                           parts_off, refs);
    else
        hipLaunchKernelGGL(k_gram_xtx<double>, dim3(nrefs), dim3(256), 0, s, ptrs, mat, m, n, rows_per_chunk, ws,
                           parts_off, refs);
    return hipGetLastError();
}

hipError_t launch_gemm(int op, int fp32, const void* const* ptrs, double* ws,
                       const GemmTask* tasks, const TileRef* tiles, int ntiles, int N,
                       hipStream_t s, const int* guard, int64_t e_part) {
    if (ntiles <= 0) return hipSuccess;
    if (op != 0 && e_part >= 0) return hipErrorInvalidValue;
    dim3 g(ntiles), b(256);
    if (N > 64 && N <= 96) {                      // one 64 x 96 tile per row strip
        if (op == 0) {
            if (fp32)
                hipLaunchKernelGGL((k_gemm_mfma<float, 0, 96, 32>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
            else
                hipLaunchKernelGGL((k_gemm_mfma<double, 0, 96, 32>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
        } else {
            if (fp32)
                hipLaunchKernelGGL((k_gemm_mfma<float, 1, 96, 32>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
            else
                hipLaunchKernelGGL((k_gemm_mfma<double, 1, 96, 32>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
        }
        return hipGetLastError();
    }
    if (op == 0) {
        if (fp32)
            hipLaunchKernelGGL((k_gemm_mfma<float, 0>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
        else
            hipLaunchKernelGGL((k_gemm_mfma<double, 0>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_gemm_mfma<float, 1>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
        else
            hipLaunchKernelGGL((k_gemm_mfma<double, 1>), g, b, 0, s, ptrs, ws, tasks, tiles, N, guard, e_part);
    }
    return hipGetLastError();
}

}  // namespace hsvd
