// Passes over A on the matrix cores, for mixed-precision plans:
//   op 0: Y = A_blk * X,   op 1: Y = A_blk^T * X,
// with A (float32, row-major) and X (float64 col-major panel) rounded to bfloat16
// (nearest even), products summed in float32 by v_mfma_f32_16x16x32_bf16, and Y
// written as float64.  These passes are bound by HBM: A is read exactly once.
//
// A 512-thread work-group owns a strip of 256 output rows and every output column
// (N <= 96, as 16-column tiles); wave w computes rows [32 w, 32 w + 32) as 2 x NT
// MFMA tiles.  The reduction streams in slabs of 64:
//   * X's slab (64 x N, float64) is read coalesced, rounded and stored in LDS as
//     [column][k] so that a lane's B operand (8 consecutive k) is one 16-byte read;
//   * op 0: a lane's A operand is 8 consecutive floats of one row of A, read straight
//     from global memory as two 16-byte loads (4 lanes cover 128 contiguous bytes);
//   * op 1: the slab of A (64 rows x 256 columns) is read as rows (16-byte loads, a
//     wave covers 1 KB of a row), transposed on the way into LDS by packing 8 rows of a
//     column into one 16-byte store, then read as A operands like X.
// Slabs are double-buffered (one barrier per slab) and the next slab's global loads
// are issued before the current slab's matrix-core work (op 0 keeps A one slab
// ahead, X two: its panel comes through L2 from other XCDs' writes).  Work-groups
// are ordered so that consecutive strips (the strips of one block, which share X) run
// on the same XCD.
//
// MFMA 16x16x32 operand layout (lane l of 64): A fragment row l % 16, reduction
// indices 8 (l / 16) .. 8 (l / 16) + 7; B fragment column l % 16, same reduction
// indices; the 4 accumulators of lane l hold column l % 16, rows 4 (l / 16) + e.
#include "hsvd_internal.hpp"
#include <type_traits>

namespace hsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int BT = 512;                 // threads
constexpr int BM = kBf16TileRows;       // output rows per strip (256)
constexpr int BK = 64;                  // reduction slab
constexpr int PK = BK + 8;              // LDS pitch (bf16) of a [row or column][k] line: 144 bytes
constexpr int NMAX = kBf16MaxN;         // output columns (96)
constexpr int XS = NMAX * PK;           // one X slab buffer (bf16)
constexpr int AS = BM * PK;             // one A slab buffer (op 1)

__device__ __forceinline__ bf16x8 to_bf16x8(const float (&v)[8]) {
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];
    return r;
}

// The tile of work-group b when the grid is split into 8 contiguous chunks, chunk x on
// XCD x (work-groups are dispatched to the XCDs round robin).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    if (n % 8) return b;
    return (b % 8) * (n / 8) + b / 8;
}

}  // namespace

template <int OP>
__global__ __launch_bounds__(BT) void k_gemm_bf16(const void* const* __restrict__ ptrs,
                                                  double* __restrict__ ws,
                                                  const GemmTask* __restrict__ tasks,
                                                  const TileRef* __restrict__ tiles, int ntiles, int N) {
    extern __shared__ __attribute__((aligned(16))) __bf16 bsm[];
    __bf16* Xs = bsm;                   // 2 buffers of [column][k]
    __bf16* As = bsm + 2 * XS;          // op 1: 2 buffers of [output row][k]
    const TileRef tr = tiles[xcd_tile(blockIdx.x, ntiles)];
    const GemmTask t = tasks[tr.task];
    const int r0 = tr.tile * BM;
    const int out_rows = OP == 0 ? t.rows : t.cols;
    const int K = OP == 0 ? t.cols : t.rows;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const float* Ab = (const float*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;
    const int NT = (N + 15) >> 4;
    const int nslab = (K + BK - 1) / BK;
    auto k_of = [&](int sl) { return sl * BK; };

    // ---- X slab: element e = (column c, k kk), kk fastest; 12 per thread at N = 96
    constexpr int XE = NMAX * BK / BT;
    double xr[XE];
    auto load_x = [&](int k0) {
#pragma unroll
        for (int u = 0; u < XE; ++u) {
            const int e = tid + BT * u, c = e / BK, kk = e % BK;
            const int gk = k0 + kk;
            xr[u] = (c < N && gk < K) ? X[(int64_t)c * t.x_ld + gk] : 0.0;
        }
    };
    auto store_x = [&](__bf16* dst) {
#pragma unroll
        for (int u = 0; u < XE; ++u) {
            const int e = tid + BT * u, c = e / BK, kk = e % BK;
            dst[c * PK + kk] = (__bf16)(float)xr[u];
        }
    };

    // ---- A operand
    // op 0: per wave 2 row tiles x 2 k-steps of 8 floats (direct fragments, below)
    // op 1: the slab of A is 64 rows x 256 columns; item (row group g of 8 rows, column
    // quad c4): one per thread (8 row groups x 64 column quads = 512), a 16-byte load per
    // row, a wave's load covering 1 KB of one row
    constexpr int AQ = BM / 4;                    // column quads of a slab row
    static_assert((BK / 8) * AQ == BT, "one op-1 item per thread");
    f32x4 at[8];
    auto load_a1 = [&](int k0) {
        const int g = tid / AQ, c4 = tid % AQ;
        const int gc = r0 + 4 * c4;               // output rows are columns of A
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int gk = k0 + 8 * g + e;
            const float* src = Ab + (int64_t)gk * lda + gc;
            f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (gk < K) {
                if (gc + 4 <= out_rows && ((uintptr_t)src & 15) == 0) v = *(const f32x4*)src;
                else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (gc + q < out_rows) v[q] = src[q];
                }
            }
            at[e] = v;
        }
    };
    auto store_a1 = [&](__bf16* dst) {
        const int g = tid / AQ, c4 = tid % AQ;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float c[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) c[e] = at[e][q];
            *(bf16x8*)&dst[(4 * c4 + q) * PK + 8 * g] = to_bf16x8(c);
        }
    };

    f32x4 acc[2][NMAX / 16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NMAX / 16; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    if constexpr (OP == 0) {
        // op 0 keeps two slabs of A in flight (A is the HBM stream; X comes from L2 and
        // stays one slab ahead): slab sl + 2 is requested while slab sl is multiplied
        float ar[2][2][8];                           // the next slab
        auto load_to = [&](float (&dst)[2][2][8], int k0) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int gr = r0 + 32 * wave + 16 * i + li;
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int gk = k0 + 32 * s2 + 8 * lq;
                    const float* src = Ab + (int64_t)gr * lda + gk;
                    if (gr < out_rows && gk + 8 <= K && ((uintptr_t)src & 15) == 0) {
                        const f32x4 v0 = *(const f32x4*)src;
                        const f32x4 v1 = *(const f32x4*)(src + 4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) { dst[i][s2][e] = v0[e]; dst[i][s2][4 + e] = v1[e]; }
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            dst[i][s2][e] = (gr < out_rows && gk + e < K) ? src[e] : 0.0f;
                    }
                }
            }
        };
        // X (from L2, one pass-wide panel) two slabs ahead, A one slab ahead
        double xq[XE];                               // X of the slab after next
        auto load_xq = [&](int k0) {
#pragma unroll
            for (int u = 0; u < XE; ++u) {
                const int e = tid + BT * u, c = e / BK, kk = e % BK;
                const int gk = k0 + kk;
                xq[u] = (c < N && gk < K) ? X[(int64_t)c * t.x_ld + gk] : 0.0;
            }
        };
        auto store_xq = [&](__bf16* dst) {
#pragma unroll
            for (int u = 0; u < XE; ++u) {
                const int e = tid + BT * u, c = e / BK, kk = e % BK;
                dst[c * PK + kk] = (__bf16)(float)xq[u];
            }
        };
        load_x(k_of(0));
        load_to(ar, k_of(0));
        store_x(Xs);
        if (nslab > 1) load_x(k_of(1));
        __syncthreads();
        auto step = [&](auto bufc, int sl) {
            constexpr int B = decltype(bufc)::value;   // xr holds slab sl + 1 when B == 0
            const __bf16* xs = Xs + (sl & 1) * XS;
            bf16x8 afr[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) afr[i][s2] = to_bf16x8(ar[i][s2]);
            if (sl + 1 < nslab) load_to(ar, k_of(sl + 1));
            if (sl + 2 < nslab) {
                if (B == 0) load_xq(k_of(sl + 2));
                else load_x(k_of(sl + 2));
            }
#pragma unroll
            for (int j = 0; j < NMAX / 16; ++j) {
                if (j < NT) {
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) {
                        const bf16x8 b = *(const bf16x8*)&xs[(16 * j + li) * PK + 32 * s2 + 8 * lq];
#pragma unroll
                        for (int i = 0; i < 2; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i][s2], b, acc[i][j], 0, 0, 0);
                    }
                }
            }
            if (sl + 1 < nslab) {
                if (B == 0) store_x(Xs + ((sl & 1) ^ 1) * XS);
                else store_xq(Xs + ((sl & 1) ^ 1) * XS);
            }
            __syncthreads();
        };
        for (int sl = 0; sl < nslab; sl += 2) {
            step(std::integral_constant<int, 0>{}, sl);
            if (sl + 1 < nslab) step(std::integral_constant<int, 1>{}, sl + 1);
        }
    } else {
    load_x(k_of(0));
    load_a1(k_of(0));
    store_x(Xs);
    store_a1(As);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const int buf = sl & 1;
        const __bf16* xs = Xs + buf * XS;
        const __bf16* as = As + buf * AS;
        bf16x8 afr[2][2];
        const bool more = sl + 1 < nslab;
        if (more) {                                  // next slab's loads in flight
            load_x(k_of(sl + 1));
            load_a1(k_of(sl + 1));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                afr[i][s] = *(const bf16x8*)&as[(32 * wave + 16 * i + li) * PK + 32 * s + 8 * lq];
#pragma unroll
        for (int j = 0; j < NMAX / 16; ++j) {
            if (j < NT) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const bf16x8 b = *(const bf16x8*)&xs[(16 * j + li) * PK + 32 * s + 8 * lq];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i][s], b, acc[i][j], 0, 0, 0);
                }
            }
        }
        if (more) {
            store_x(Xs + (buf ^ 1) * XS);
            store_a1(As + (buf ^ 1) * AS);
        }
        __syncthreads();
    }
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < NMAX / 16; ++j) {
        const int gc = 16 * j + li;
        if (j >= NT || gc >= N) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int gr = r0 + 32 * wave + 16 * i + 4 * lq;
            double* dst = Y + (int64_t)gc * t.y_ld + gr;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (gr + e < out_rows) dst[e] = (double)acc[i][j][e];
        }
    }
}

hipError_t prepare_gemm_bf16_launches() {
    static unsigned long long d0 = 0, d1 = 0;
    hipError_t e = set_lds_limit_once((const void*)k_gemm_bf16<0>, (int)(sizeof(__bf16) * (size_t)(2 * XS + 2 * AS)), &d0);
    if (e == hipSuccess) e = set_lds_limit_once((const void*)k_gemm_bf16<1>, (int)(sizeof(__bf16) * (size_t)(2 * XS + 2 * AS)), &d1);
    return e;
}

hipError_t launch_gemm_bf16(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                            const TileRef* tiles, int ntiles, int N, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (N < 1 || N > NMAX) return hipErrorInvalidValue;
    const size_t lds = sizeof(__bf16) * (size_t)(2 * XS + (op == 1 ? 2 * AS : 0));
    hipError_t e = prepare_gemm_bf16_launches();
    if (e != hipSuccess) return e;
    dim3 g(ntiles), b(BT);
    if (op == 0) {
        hipLaunchKernelGGL(k_gemm_bf16<0>, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    } else {
        hipLaunchKernelGGL(k_gemm_bf16<1>, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    }
    return hipGetLastError();
}

}  // namespace hsvd
