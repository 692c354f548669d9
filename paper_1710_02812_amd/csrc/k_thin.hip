// Thin-panel algebra on col-major float64 panels, split into row chunks so that
// every level of the merge tree keeps many work-groups busy:
//   gram   : part[c] = X_c^T Y_c                    (projection coefficients, CGS)
//   reduce : C = sum_c part[c];  Cacc = C or Cacc += C (one group per task)
//   nn     : Y_c = X_c C  |  Y_c += X_c C  |  Y_c -= X_c C
//   sum    : Y_c = sum_j P_j,c (partial products of a split reduction)
// Widths are at most 128; gram and nn run one 64 x 64 output tile per group on the
// float64 matrix cores.
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

constexpr int TT = MF_T;
constexpr int TK = 32;          // slab depth: the reductions here are short (panel widths)

// part (wx x wy) = X_c^T Y_c for one chunk on the float64 matrix cores; grid: chunk x
// (wx / 64) x (wy / 64) tiles.  X_c^T is a row-major wx x rows array (leading
// dimension x_ld), Y_c a column-major rows x wy panel.
__global__ __launch_bounds__(256) void k_thin_gram(double* __restrict__ ws,
                                                   const ThinTask* __restrict__ tasks,
                                                   const ChunkRef* __restrict__ chunks, int chh) {
    __shared__ double As[mfma_lds_a<0, TK>()];
    __shared__ double Bs[mfma_lds_b<TK>()];
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int bx = blockIdx.y * TT, by = blockIdx.z * TT;
    if (bx >= t.wx || by >= t.wy) return;
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    v4d acc[2][2];
    mfma_tile<double, 0, true, double, false, false, TK>(ws + t.x_off + row0, t.x_ld, ws + t.y_off + row0, t.y_ld,
                                                        t.wx, t.wy, rows, bx, by, As, Bs, acc);
    double* P = ws + t.part_off + (int64_t)cr.chunk * t.wx * t.wy;
    mfma_tile_out(t.wx, t.wy, bx, by, acc, [&](int r, int c, double v) { P[(int64_t)c * t.wx + r] = v; });
}

__global__ __launch_bounds__(256) void k_thin_reduce(double* __restrict__ ws,
                                                     const ThinTask* __restrict__ tasks) {
    // grid: task x (element slices of 256); one thread per element of C, partials
    // summed in chunk order
    const ThinTask t = tasks[blockIdx.x];
    const int64_t sz = (int64_t)t.wx * t.wy;
    const int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= sz) return;
    const double* P = ws + t.part_off + e;
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= t.nch; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)(c + u) * sz];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < t.nch; ++c) s += P[(int64_t)c * sz];
    const int j = (int)(e / t.wx), i = (int)(e - (int64_t)j * t.wx);
    ws[t.c_off + (int64_t)j * t.c_ld + i] = s;
    if (t.acc_off >= 0) {
        double* a = ws + t.acc_off + (int64_t)j * t.c_ld + i;
        *a = t.accumulate ? *a + s : s;
    }
}

// Y_c (op)= X_c * C with C (wx x wy, ld c_ld) on the float64 matrix cores; grid: chunk
// x (chh / 64) row tiles x (wy / 64) column tiles.  X_c (rows x wx, column-major) is the
// transpose of a row-major wx x rows array.
// Three work-groups per CU: the register cap costs one spilled register (a 4-byte
// store and reload) and shortens the Q updates of a merge level by about a tenth.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_thin_nn(double* __restrict__ ws, const int* __restrict__ iws,
                                                 const ThinTask* __restrict__ tasks,
                                                 const ChunkRef* __restrict__ chunks, int chh) {
    __shared__ double As[MF_T * (MF_T + 1)];     // the A slabs, then the output tile
    __shared__ double Bs[mfma_lds_b<TK>()];
    static_assert(mfma_lds_a<1, TK>() <= MF_T * (MF_T + 1), "A staging");
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int rt = blockIdx.y * TT, by = blockIdx.z * TT;
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    if (rt >= rows || by >= t.wy) return;
    if (t.cond >= 0 && iws[t.cond] != 0) return;
    v4d acc[2][2];
    mfma_tile<double, 1, true, double, false, false, TK>(ws + t.x_off + row0, t.x_ld, ws + t.c_off, t.c_ld, rows,
                                                        t.wy, t.wx, rt, by, As, Bs, acc);
    if (t.x2_off >= 0)
        mfma_tile<double, 1, false, double, false, false, TK>(ws + t.x2_off + row0, t.x2_ld, ws + t.c2_off, t.c2_ld,
                                                             rows, t.wy, t.wx2, rt, by, As, Bs, acc);
    double* Y = ws + t.y_off + row0;
    const int mode = t.accumulate;
    mfma_tile_out_lds(rows, t.wy, rt, by, acc, As, [&](int r, int c, double v) {
        double* y = Y + (int64_t)c * t.y_ld + r;
        if (mode == 0) *y = v;
        else if (mode == 1) *y += v;
        else *y -= v;
    });
}

// Y_c = sum_{j < wx} P_j,c with P_j = X + j * c_ld (each ld x_ld), width wy; grid:
// chunk x column, one thread per row (the partials summed in order j = 0, 1, ...).
__global__ __launch_bounds__(256) void k_thin_sum(double* __restrict__ ws,
                                                  const ThinTask* __restrict__ tasks,
                                                  const ChunkRef* __restrict__ chunks, int chh) {
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int c = blockIdx.y;
    if (c >= t.wy) return;
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    const double* X = ws + t.x_off + (int64_t)c * t.x_ld + row0;
    double* Y = ws + t.y_off + (int64_t)c * t.y_ld + row0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        double s = 0.0;
        int j = 0;
        for (; j + 4 <= t.wx; j += 4) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = X[(int64_t)(j + u) * t.c_ld + r];
#pragma unroll
            for (int u = 0; u < 4; ++u) s += v[u];
        }
        for (; j < t.wx; ++j) s += X[(int64_t)j * t.c_ld + r];
        Y[r] = s;
    }
}

hipError_t launch_thin_gram(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                            int chh, hipStream_t s, int tx, int ty) {
    if (nchunks <= 0) return hipSuccess;
    if (tx < 1 || tx > 2 || ty < 1 || ty > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_thin_gram, dim3(nchunks, tx, ty), dim3(256), 0, s, ws, t, chunks, chh);
    return hipGetLastError();
}
hipError_t launch_thin_reduce(double* ws, const ThinTask* t, int ntasks, int maxsz, hipStream_t s) {
    if (ntasks <= 0 || maxsz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_reduce, dim3(ntasks, (maxsz + 255) / 256), dim3(256), 0, s, ws, t);
    return hipGetLastError();
}
hipError_t launch_thin_nn(double* ws, const int* iws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                          int chh, hipStream_t s, int ty) {
    if (nchunks <= 0) return hipSuccess;
    if (ty < 1 || ty > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_thin_nn, dim3(nchunks, (chh + TT - 1) / TT, ty), dim3(256), 0, s, ws, iws, t, chunks, chh);
    return hipGetLastError();
}
hipError_t launch_thin_sum(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                           int chh, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_sum, dim3(nchunks, 128), dim3(256), 0, s, ws, t, chunks, chh);
    return hipGetLastError();
}

}  // namespace hsvd
