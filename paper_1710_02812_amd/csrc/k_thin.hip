// Thin-panel algebra on col-major float64 panels, split into row chunks so that
// every level of the merge tree keeps many work-groups busy:
//   gram   : part[c] = X_c^T Y_c                    (projection coefficients, CGS)
//   reduce : C = sum_c part[c];  Cacc = C or Cacc += C (one group per task)
//   nn     : Y_c = X_c C  |  Y_c += X_c C  |  Y_c -= X_c C
//   sum    : Y_c = sum_j P_j,c (partial products of a split reduction)
// Widths are at most 128; a group handles a 64-row x 64-column output tile.
#include "hsvd_internal.hpp"
#include "device_common.hpp"

namespace hsvd {

constexpr int TT = 64;

// part (wx x wy) = X_c^T Y_c for one chunk; grid: chunk x (wx/64) x (wy/64) tiles.
__global__ __launch_bounds__(256) void k_thin_gram(double* __restrict__ ws,
                                                   const ThinTask* __restrict__ tasks,
                                                   const ChunkRef* __restrict__ chunks, int chh) {
    __shared__ double Xs[32][TT + 1];
    __shared__ double Ys[32][TT + 1];
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int bx = blockIdx.y * TT, by = blockIdx.z * TT;
    if (bx >= t.wx || by >= t.wy) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    const double* X = ws + t.x_off + row0;
    const double* Y = ws + t.y_off + row0;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < rows; k0 += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int c = e >> 5, kk = e & 31;
            const bool ok = (k0 + kk) < rows;
            Xs[kk][c] = (ok && bx + c < t.wx) ? X[(int64_t)(bx + c) * t.x_ld + k0 + kk] : 0.0;
            Ys[kk][c] = (ok && by + c < t.wy) ? Y[(int64_t)(by + c) * t.y_ld + k0 + kk] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Xs[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Ys[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* P = ws + t.part_off + (int64_t)cr.chunk * t.wx * t.wy;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = bx + ty + 16 * i, c = by + tx + 16 * j;
            if (r < t.wx && c < t.wy) P[(int64_t)c * t.wx + r] = acc[i][j];
        }
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

// Y_c (op)= X_c * C  with C (wx x wy, ld c_ld); grid: chunk x (wy/64) column tiles.
__global__ __launch_bounds__(256) void k_thin_nn(double* __restrict__ ws,
                                                 const ThinTask* __restrict__ tasks,
                                                 const ChunkRef* __restrict__ chunks, int chh) {
    __shared__ double Cs[128][TT + 1];   // [l][col]
    __shared__ double Xs[TT][129];       // [row][l]
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int by = blockIdx.y * TT;
    if (by >= t.wy) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    const double* C = ws + t.c_off;
    for (int e = tid; e < t.wx * TT; e += 256) {
        const int c = e / t.wx, l = e - c * t.wx;
        Cs[l][c] = (by + c < t.wy) ? C[(int64_t)(by + c) * t.c_ld + l] : 0.0;
    }
    const double* X = ws + t.x_off;
    double* Y = ws + t.y_off;
    for (int r0 = 0; r0 < rows; r0 += TT) {
        __syncthreads();
        for (int e = tid; e < t.wx * TT; e += 256) {
            const int l = e / TT, r = e - l * TT;
            Xs[r][l] = (r0 + r < rows) ? X[(int64_t)l * t.x_ld + row0 + r0 + r] : 0.0;
        }
        __syncthreads();
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int l = 0; l < t.wx; ++l) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Xs[ty + 16 * i][l];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Cs[l][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + ty + 16 * i, c = by + tx + 16 * j;
                if (r < rows && c < t.wy) {
                    double* y = Y + (int64_t)c * t.y_ld + row0 + r;
                    if (t.accumulate == 0) *y = acc[i][j];
                    else if (t.accumulate == 1) *y += acc[i][j];
                    else *y -= acc[i][j];
                }
            }
    }
}

// Y_c = sum_{j < wx} P_j,c with P_j = X + j * c_ld (each ld x_ld), width wy.
__global__ __launch_bounds__(256) void k_thin_sum(double* __restrict__ ws,
                                                  const ThinTask* __restrict__ tasks,
                                                  const ChunkRef* __restrict__ chunks, int chh) {
    const ChunkRef cr = chunks[blockIdx.x];
    const ThinTask t = tasks[cr.task];
    const int row0 = cr.chunk * chh;
    const int rows = min(chh, t.h - row0);
    const double* X = ws + t.x_off;
    double* Y = ws + t.y_off;
    for (int e = threadIdx.x; e < rows * t.wy; e += blockDim.x) {
        const int c = e / rows, r = e - c * rows;
        double s = 0.0;
        for (int j = 0; j < t.wx; ++j) s += X[(int64_t)j * t.c_ld + (int64_t)c * t.x_ld + row0 + r];
        Y[(int64_t)c * t.y_ld + row0 + r] = s;
    }
}

hipError_t launch_thin_gram(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                            int chh, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_gram, dim3(nchunks, 2, 2), dim3(256), 0, s, ws, t, chunks, chh);
    return hipGetLastError();
}
hipError_t launch_thin_reduce(double* ws, const ThinTask* t, int ntasks, int maxsz, hipStream_t s) {
    if (ntasks <= 0 || maxsz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_reduce, dim3(ntasks, (maxsz + 255) / 256), dim3(256), 0, s, ws, t);
    return hipGetLastError();
}
hipError_t launch_thin_nn(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                          int chh, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_nn, dim3(nchunks, 2), dim3(256), 0, s, ws, t, chunks, chh);
    return hipGetLastError();
}
hipError_t launch_thin_sub(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                           int chh, hipStream_t s) {
    return launch_thin_nn(ws, t, chunks, nchunks, chh, s);
}
hipError_t launch_thin_sum(double* ws, const ThinTask* t, const ChunkRef* chunks, int nchunks,
                           int chh, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_sum, dim3(nchunks), dim3(256), 0, s, ws, t, chunks, chh);
    return hipGetLastError();
}

}  // namespace hsvd
