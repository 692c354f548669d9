// One 64 x 64 output tile of a float64 product on the matrix cores
// (v_mfma_f64_16x16x4_f64), for 256-thread work-groups.  Shared by the passes over
// the input and the thin-panel kernels.
//
// C[r0 + i][c0 + j] = sum_k A(r0 + i, k) B(k, c0 + j), i, j < 64, k < K, with
//   OP 0: A row-major M x K   (A(i, k) = A[i * lda + k]),
//   OP 1: A stored K x M      (A(i, k) = A[k * lda + i], the transpose of a row-major array),
//   B column-major K x N      (B(k, j) = B[j * ldb + k]).
// Wave w owns the 32 x 32 quarter (rows 32 (w & 1), columns 32 (w >> 1)) as 2 x 2
// blocks of 16 x 16.  Per 4-deep step lane l holds A[i = l % 16][k = l / 16] and
// B[k = l / 16][j = l % 16]; accumulator element v holds C[i = l / 16 + 4 v][j = l % 16].
// Slabs of MF_K along K are staged through LDS in the order they are read from memory
// (conflict-free stores) while the next slab is fetched into registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsvd {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int MF_T = 64;        // tile rows and columns
constexpr int MF_K = 64;        // reduction slab

// LDS doubles of the staging buffers (slabs of KS along K): A slab then B slab
template <int OP, int KS = MF_K>
__host__ __device__ constexpr int mfma_lds_a() { return OP == 0 ? MF_T * (KS + 1) : KS * (MF_T + 1); }
template <int KS = MF_K, int NC = MF_T>
__host__ __device__ constexpr int mfma_lds_b() { return NC * (KS + 1); }

// With ZERO false the products add to acc as it stands (a second operand pair).
// TB / BROW: B's element type and layout (BROW: B row-major, B(k, j) = B[k * ldb + j],
// read with consecutive threads on consecutive columns).
// SQ: *ssq (per thread) accumulates the squares of the A elements this thread stages
// (over the work-group: the squared Frobenius norm of the tile's rows of A, OP 0).
// KS: the slab depth (64, or 32 for short reductions: half the staging registers and
// LDS, so that more work-groups share a compute unit).
// NC: the tile's columns, 64 or 96 (a 64 x 96 tile: wave w owns rows 32 (w & 1) and
// columns 48 (w >> 1) as 2 x 3 blocks, so that a product up to 96 columns wide reads
// its A once).
template <typename TA, int OP, bool ZERO = true, typename TB = double, bool BROW = false, bool SQ = false,
          int KS = MF_K, int NC = MF_T>
__device__ __forceinline__ void mfma_tile(const TA* __restrict__ A, int64_t lda,
                                          const TB* __restrict__ B, int64_t ldb,
                                          int M, int N, int K, int r0, int c0, double* As, double* Bs,
                                          v4d (&acc)[2][NC / 32], double* ssq = nullptr) {
    static_assert(NC == 64 || NC == 96, "tile columns");
    constexpr int NJ = NC / 32;                              // column blocks per wave
    constexpr int AP = OP == 0 ? KS + 1 : MF_T + 1;
    constexpr int BP = KS + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * (NC / 2);
    const int li = lane & 15, lk = lane >> 4;
    constexpr int NE = MF_T * KS / 256;                      // A slab elements per thread
    constexpr int NEB = NC * KS / 256;                       // B slab elements per thread
    TA pa[NE];
    TB pb[NEB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            if (OP == 0) {
                const int r = e / KS, kk = e % KS;        // A(r0 + r, k0 + kk)
                const int gr = r0 + r, gk = k0 + kk;
                pa[u] = (gr < M && gk < K) ? A[(int64_t)gr * lda + gk] : (TA)0;
            } else {
                const int kk = e / MF_T, c = e % MF_T;        // A(r0 + c, k0 + kk)
                const int gk = k0 + kk, gc = r0 + c;
                pa[u] = (gk < K && gc < M) ? A[(int64_t)gk * lda + gc] : (TA)0;
            }
        }
#pragma unroll
        for (int u = 0; u < NEB; ++u) {
            const int e = tid + 256 * u;
            const int bc = BROW ? e % NC : e / KS, bk = BROW ? e / NC : e % KS;   // B(k0 + bk, c0 + bc)
            const int gbc = c0 + bc, gbk = k0 + bk;
            if (BROW) pb[u] = (gbc < N && gbk < K) ? B[(int64_t)gbk * ldb + gbc] : (TB)0;
            else pb[u] = (gbc < N && gbk < K) ? B[(int64_t)gbc * ldb + gbk] : (TB)0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            if constexpr (SQ) *ssq = fma((double)pa[u], (double)pa[u], *ssq);
            if (OP == 0) As[(e / KS) * AP + (e % KS)] = (double)pa[u];
            else As[(e / MF_T) * AP + (e % MF_T)] = (double)pa[u];
        }
#pragma unroll
        for (int u = 0; u < NEB; ++u) {
            const int e = tid + 256 * u;
            if (BROW) Bs[(e % NC) * BP + (e / NC)] = (double)pb[u];
            else Bs[(e / KS) * BP + (e % KS)] = (double)pb[u];
        }
    };
    if (ZERO)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KS) {
        stage();
        __syncthreads();
        if (k0 + KS < K) fetch(k0 + KS);                  // in flight during the products
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {
            const int kk = 4 * q + lk;
            double a[2], b[NJ];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wr + 16 * i + li;
                a[i] = OP == 0 ? As[row * AP + kk] : As[kk * AP + row];
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) b[j] = Bs[(wc + 16 * j + li) * BP + kk];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
}

// Visits the tile's outputs: f(row, col, value) for rows < M, columns < N.
template <typename F, int NJ>
__device__ __forceinline__ void mfma_tile_out(int M, int N, int r0, int c0, const v4d (&acc)[2][NJ], F f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * (16 * NJ);    // NJ = tile columns / 32
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int gc = c0 + wc + 16 * j + li;
        if (gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = r0 + wr + 16 * i + lk + 4 * v;
                if (gr < M) f(gr, gc, acc[i][j][v]);
            }
    }
}

// mfma_tile_out with coalesced stores: the tile goes through buf (>= 64 x 65 doubles of
// LDS, free after mfma_tile, which ends on a barrier), then wave w visits columns
// w, w + 4, ... with lane l on row l, so each column's 64 rows are one contiguous run.
// Every thread of the 256 calls it; it ends on a barrier (buf may be reused after).
template <typename F>
__device__ __forceinline__ void mfma_tile_out_lds(int M, int N, int r0, int c0, const v4d (&acc)[2][2],
                                                  double* buf, F f) {
    constexpr int LD = MF_T + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                buf[(wc + 16 * j + li) * LD + wr + 16 * i + lk + 4 * v] = acc[i][j][v];
    __syncthreads();
    const int gr = r0 + lane;
    if (gr < M)
        for (int c = wave; c < MF_T; c += 4) {
            const int gc = c0 + c;
            if (gc < N) f(gr, gc, buf[c * LD + lane]);
        }
    __syncthreads();
}

// A small product whose operands are already on chip: C (M x N) = A (M x K) B (K x N)
// with a(i, k) and b(k, j) reading LDS (or cached global) elements; 16 x 16 output
// tiles are dealt to the waves of the work-group (tile t to wave t mod nw), each a
// chain of K / 4 matrix-core steps with one operand value per lane.  Reads are
// clamped into range and zeroed outside it (no branch between the loads).
// out(i, j, v) receives each element (i < M, j < N).
template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void mfma_small(int M, int N, int K, FA a, FB b, FO out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (M + 15) / 16, tn = (N + 15) / 16;
    for (int t = wave; t < tm * tn; t += nw) {
        const int i0 = (t % tm) * 16, j0 = (t / tm) * 16;
        const int ia = min(i0 + li, M - 1), jb = min(j0 + li, N - 1);
        const bool iok = i0 + li < M, jok = j0 + li < N;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk, kc = min(k, K - 1);
            const double av = a(ia, kc), bv = b(kc, jb);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((iok && k < K) ? av : 0.0,
                                                       (jok && k < K) ? bv : 0.0, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + lk + 4 * v;
            if (i < M && jok) out(i, j0 + li, acc[v]);
        }
    }
}

// mfma_small for in-place products: the wave's tiles t = wave + nw u (u < NT; the
// caller checks that tm tn <= NT nw) are computed into acc, to be written with
// mfma_small_store after a barrier.
template <int NT, typename FA, typename FB>
__device__ __forceinline__ void mfma_small_keep(int M, int N, int K, FA a, FB b, v4d (&acc)[NT]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (M + 15) / 16, tn = (N + 15) / 16;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
        const int t = wave + nw * u;
        if (t >= tm * tn) continue;
        const int i0 = (t % tm) * 16, j0 = (t / tm) * 16;
        const int ia = min(i0 + li, M - 1), jb = min(j0 + li, N - 1);
        const bool iok = i0 + li < M, jok = j0 + li < N;
#pragma unroll 4
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk, kc = min(k, K - 1);
            const double av = a(ia, kc), bv = b(kc, jb);
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((iok && k < K) ? av : 0.0,
                                                          (jok && k < K) ? bv : 0.0, acc[u], 0, 0, 0);
        }
    }
}
template <int NT, typename FO>
__device__ __forceinline__ void mfma_small_store(int M, int N, const v4d (&acc)[NT], FO out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (M + 15) / 16, tn = (N + 15) / 16;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int t = wave + nw * u;
        if (t >= tm * tn) continue;
        const int i0 = (t % tm) * 16, j = (t / tm) * 16 + li;
        if (j >= N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + lk + 4 * v;
            if (i < M) out(i, j, acc[u][v]);
        }
    }
}

}  // namespace hsvd
