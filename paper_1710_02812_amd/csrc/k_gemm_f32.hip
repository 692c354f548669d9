// Passes over A on the float32 matrix cores, for the mixed-precision plans' products
// that must be float32-accurate (the projection Y = A V and Algorithm 2's W = U^T A):
//   op 0: Y = A_blk * X,   op 1: Y = A_blk^T * X,
// with A (float32, row-major) exact, X (float64 col-major panel) rounded to float32,
// products and sums in float32 (v_mfma_f32_16x16x4_f32), Y written as float64.
//
// The layout follows the bfloat16 passes: a 512-thread work-group owns a strip of 256
// output rows and every output column (N <= 96); wave w computes rows [32 w, 32 w + 32)
// as 2 x NT tiles of 16 x 16.  The reduction streams in slabs of 32 through LDS,
// double-buffered with one barrier per slab, the next slab's global loads issued before
// the current slab's matrix-core work:
//   * X's slab (32 x N) as [column][k], pitch 36 floats;
//   * op 0: A's slab (256 rows x 32) as [row][k], pitch 36 (16-byte row loads);
//   * op 1: A's slab (32 rows x 256 columns) as stored, [k][column], pitch 272.
// Per 4-deep step lane l holds A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16];
// both pitches put the 64 lanes of a read on distinct banks.  Accumulator element e of
// lane l holds C[i = 4 (l / 16) + e][j = l % 16].
#include "hsvd_internal.hpp"
#include <type_traits>

namespace hsvd {

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int FT = 512;                 // threads
constexpr int FM = kBf16TileRows;       // output rows per strip (256)
constexpr int FK = 32;                  // reduction slab
constexpr int PX = FK + 4;              // [column][k] and [row][k] pitch (floats)
constexpr int PT = FM + 16;             // [k][column] pitch (floats)
constexpr int FN = kBf16MaxN;           // output columns (96)
constexpr int XSZ = FN * PX;
constexpr int ASZ = (FM * PX > FK * PT) ? FM * PX : FK * PT;

__device__ __forceinline__ int xcd_tile32(int b, int n) {
    if (n % 8) return b;
    return (b % 8) * (n / 8) + b / 8;
}

}  // namespace

template <int OP>
__global__ __launch_bounds__(FT) void k_gemm_f32(const void* const* __restrict__ ptrs,
                                                 double* __restrict__ ws,
                                                 const GemmTask* __restrict__ tasks,
                                                 const TileRef* __restrict__ tiles, int ntiles, int N) {
    extern __shared__ __attribute__((aligned(16))) float fsm[];
    float* Xs = fsm;                    // 2 buffers
    float* As = fsm + 2 * XSZ;          // 2 buffers
    const TileRef tr = tiles[xcd_tile32(blockIdx.x, ntiles)];
    const GemmTask t = tasks[tr.task];
    const int r0 = tr.tile * FM;
    const int out_rows = OP == 0 ? t.rows : t.cols;
    const int K = OP == 0 ? t.cols : t.rows;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const float* Ab = (const float*)ptrs[4 * t.mat] + t.a_off;
    const int64_t lda = t.lda;
    const double* X = ws + t.x_off;
    const int NT = (N + 15) >> 4;
    const int nslab = (K + FK - 1) / FK;
    auto k_of = [&](int sl) { return sl * FK; };

    // Two slabs of A and X are in flight at once (registers hold slab sl + 1 and slab
    // sl + 2 while slab sl is multiplied out of LDS): one slab's loads cover less than
    // the loaded-memory latency at full bandwidth.
    // X slab: 32 x 96 elements, 6 per thread, k fastest
    constexpr int XE = FN * FK / FT;
    auto load_x = [&](double (&xr)[XE], int k0) {
#pragma unroll
        for (int u = 0; u < XE; ++u) {
            const int e = tid + FT * u, c = e / FK, kk = e % FK;
            const int gk = k0 + kk;
            xr[u] = (c < N && gk < K) ? X[(int64_t)c * t.x_ld + gk] : 0.0;
        }
    };
    auto store_x = [&](const double (&xr)[XE], float* dst) {
#pragma unroll
        for (int u = 0; u < XE; ++u) {
            const int e = tid + FT * u, c = e / FK, kk = e % FK;
            dst[c * PX + kk] = (float)xr[u];
        }
    };
    // A slab: 256 x 32 floats = 2048 float4, 4 per thread
    constexpr int AE = FM * FK / 4 / FT;
    auto load_a = [&](f32x4 (&ar)[AE], int k0) {
#pragma unroll
        for (int u = 0; u < AE; ++u) {
            const int e = tid + FT * u;
            int row, col;                         // as stored in A: element (row, col .. col + 3)
            if (OP == 0) { row = r0 + e / (FK / 4); col = k0 + 4 * (e % (FK / 4)); }
            else { row = k0 + e / (FM / 4); col = r0 + 4 * (e % (FM / 4)); }
            const int rlim = OP == 0 ? out_rows : K, clim = OP == 0 ? K : out_rows;
            const float* src = Ab + (int64_t)row * lda + col;
            f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (row < rlim) {
                if (col + 4 <= clim && ((uintptr_t)src & 15) == 0) v = *(const f32x4*)src;
                else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (col + q < clim) v[q] = src[q];
                }
            }
            ar[u] = v;
        }
    };
    auto store_a = [&](const f32x4 (&ar)[AE], float* dst) {
#pragma unroll
        for (int u = 0; u < AE; ++u) {
            const int e = tid + FT * u;
            if (OP == 0) *(f32x4*)&dst[(e / (FK / 4)) * PX + 4 * (e % (FK / 4))] = ar[u];
            else *(f32x4*)&dst[(e / (FM / 4)) * PT + 4 * (e % (FM / 4))] = ar[u];
        }
    };

    f32x4 acc[2][FN / 16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN / 16; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    double x0[XE], x1[XE];                      // X of slabs in flight (alternating)
    f32x4 a0[AE], a1[AE];                       // A likewise
    load_x(x0, k_of(0));
    load_a(a0, k_of(0));
    if (nslab > 1) {
        load_x(x1, k_of(1));
        load_a(a1, k_of(1));
    }
    store_x(x0, Xs);
    store_a(a0, As);
    __syncthreads();
    // step sl: LDS buffer sl & 1 holds slab sl; registers set (sl + 1) & 1 hold slab sl + 1;
    // the set sl & 1 (slab sl, already in LDS) is refilled with slab sl + 2
    auto step = [&](auto setc, int sl) {
        constexpr int B = decltype(setc)::value;
        double (&xn)[XE] = B == 0 ? x0 : x1;
        f32x4 (&an)[AE] = B == 0 ? a0 : a1;
        const double (&xh)[XE] = B == 0 ? x1 : x0;
        const f32x4 (&ah)[AE] = B == 0 ? a1 : a0;
        const float* xs = Xs + B * XSZ;
        const float* as = As + B * ASZ;
        if (sl + 2 < nslab) {
            load_x(xn, k_of(sl + 2));
            load_a(an, k_of(sl + 2));
        }
#pragma unroll
        for (int ks = 0; ks < FK / 4; ++ks) {
            const int kk = 4 * ks + lq;
            float a[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = 32 * wave + 16 * i + li;
                a[i] = OP == 0 ? as[row * PX + kk] : as[kk * PT + row];
            }
#pragma unroll
            for (int j = 0; j < FN / 16; ++j) {
                if (j < NT) {
                    const float b = xs[(16 * j + li) * PX + kk];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[i][j], 0, 0, 0);
                }
            }
        }
        if (sl + 1 < nslab) {
            store_x(xh, Xs + (B ^ 1) * XSZ);
            store_a(ah, As + (B ^ 1) * ASZ);
        }
        __syncthreads();
    };
    for (int sl = 0; sl < nslab; sl += 2) {
        step(std::integral_constant<int, 0>{}, sl);
        if (sl + 1 < nslab) step(std::integral_constant<int, 1>{}, sl + 1);
    }
    double* Y = ws + t.y_off;
#pragma unroll
    for (int j = 0; j < FN / 16; ++j) {
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

hipError_t prepare_gemm_f32_launches() {
    static unsigned long long d0 = 0, d1 = 0;
    hipError_t e = set_lds_limit_once((const void*)k_gemm_f32<0>, (int)(sizeof(float) * (size_t)(2 * XSZ + 2 * ASZ)), &d0);
    if (e == hipSuccess) e = set_lds_limit_once((const void*)k_gemm_f32<1>, (int)(sizeof(float) * (size_t)(2 * XSZ + 2 * ASZ)), &d1);
    return e;
}

hipError_t launch_gemm_f32(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                           const TileRef* tiles, int ntiles, int N, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (N < 1 || N > FN) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)(2 * XSZ + 2 * ASZ);
    hipError_t e = prepare_gemm_f32_launches();
    if (e != hipSuccess) return e;
    dim3 g(ntiles), b(FT);
    if (op == 0) {
        hipLaunchKernelGGL(k_gemm_f32<0>, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    } else {
        hipLaunchKernelGGL(k_gemm_f32<1>, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    }
    return hipGetLastError();
}

}  // namespace hsvd
