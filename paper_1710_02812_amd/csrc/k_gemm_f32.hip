// Passes over A on the float32 matrix cores, for the mixed-precision plans' products
// that must be float32-accurate (the projection Y = A V and Algorithm 2's W = U^T A):
//   op 0: Y = A_blk * X,   op 1: Y = A_blk^T * X,
// with A (float32, row-major) exact, X (float64 col-major panel) rounded to float32,
// products and sums in float32 (v_mfma_f32_16x16x4_f32), Y written as float64.
//
// The layout follows the bfloat16 passes: a 512-thread work-group owns a strip of 256
// output rows and every output column (N <= 96); wave w computes rows [32 w, 32 w + 32)
// as 2 x NT tiles of 16 x 16.  The reduction streams in slabs of 32: X's slab (32 x N)
// through LDS as [column][k] (pitch 36 floats), double-buffered with one barrier per
// slab; A's operands straight from memory into registers, one slab ahead.  The
// reduction index of a slab's 8 four-deep steps is remapped so that lane l (li = l % 16,
// lq = l / 16) covers k = 8 lq .. 8 lq + 7 (step s: k = 8 lq + s): its A values are 8
// consecutive floats of one row (op 0: two 16-byte loads) or 8 consecutive rows of one
// column (op 1: a wave's load covers 4 rows x 64 bytes, the wave's two tiles whole
// 128-byte lines), its B values 8 consecutive k of X's column (two 16-byte LDS reads);
// every k of the slab still meets its row of A and column of X once.  Accumulator
// element e of lane l holds C[i = 4 (l / 16) + e][j = l % 16].  With only X in LDS,
// op 0 fits 128 registers and two work-groups share a CU.
#include "hsvd_internal.hpp"

namespace hsvd {

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int FT = 512;                 // threads
constexpr int FM = kBf16TileRows;       // output rows per strip (256)
constexpr int FK = 32;                  // reduction slab
constexpr int PX = FK + 4;              // X's [column][k] pitch (floats)
constexpr int FN = kBf16MaxN;           // output columns (96)
constexpr int XSZ = FN * PX;

__device__ __forceinline__ int xcd_tile32(int b, int n) {
    if (n % 8) return b;
    return (b % 8) * (n / 8) + b / 8;
}

}  // namespace

template <int OP>
__device__ __forceinline__ void gemm_f32_body(const void* const* __restrict__ ptrs, double* __restrict__ ws,
                                              const GemmTask* __restrict__ tasks,
                                              const TileRef* __restrict__ tiles, int ntiles, int N) {
    extern __shared__ __attribute__((aligned(16))) float fsm[];
    float* Xs = fsm;                    // 2 buffers
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
    f32x4 acc[2][FN / 16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN / 16; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    {
        auto load_ad = [&](float (&dst)[2][8], int k0) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int gr = r0 + 32 * wave + 16 * i + li;
                const int gk = k0 + 8 * lq;
                if (OP == 0) {                  // row gr of A, 8 consecutive floats
                    const float* src = Ab + (int64_t)(gr < out_rows ? gr : 0) * lda + gk;
                    if (gr < out_rows && gk + 8 <= K && ((uintptr_t)src & 15) == 0) {
                        const f32x4 v0 = *(const f32x4*)src;
                        const f32x4 v1 = *(const f32x4*)(src + 4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) { dst[i][e] = v0[e]; dst[i][4 + e] = v1[e]; }
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) dst[i][e] = (gr < out_rows && gk + e < K) ? src[e] : 0.0f;
                    }
                } else {                        // column gr of A, 8 consecutive rows (a wave's
                                                // load covers 4 rows x 64 bytes)
                    const float* src = Ab + (int64_t)gk * lda + (gr < out_rows ? gr : 0);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        dst[i][e] = (gr < out_rows && gk + e < K) ? src[(int64_t)e * lda] : 0.0f;
                }
            }
        };
        double xr[XE];
        float ac[2][8], an[2][8];
        load_x(xr, k_of(0));
        load_ad(ac, k_of(0));
        store_x(xr, Xs);
        __syncthreads();
        for (int sl = 0; sl < nslab; ++sl) {
            const float* xs = Xs + (sl & 1) * XSZ;
            const bool more = sl + 1 < nslab;
            if (more) {
                load_x(xr, k_of(sl + 1));
                load_ad(an, k_of(sl + 1));
            }
#pragma unroll
            for (int j = 0; j < FN / 16; ++j) {
                if (j < NT) {
                    const float* xb = xs + (16 * j + li) * PX + 8 * lq;
                    const f32x4 b0 = *(const f32x4*)xb;
                    const f32x4 b1 = *(const f32x4*)(xb + 4);
#pragma unroll
                    for (int st = 0; st < 8; ++st) {
                        const float b = st < 4 ? b0[st] : b1[st - 4];
#pragma unroll
                        for (int i = 0; i < 2; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[i][st], b, acc[i][j], 0, 0, 0);
                    }
                }
            }
            if (more) {
                store_x(xr, Xs + ((sl & 1) ^ 1) * XSZ);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int e = 0; e < 8; ++e) ac[i][e] = an[i][e];
            }
            __syncthreads();
        }
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

// op 0 fits 128 registers (two work-groups per CU); op 1's strided column loads need
// more (capped at 128 they spill), so it keeps the looser bound
__global__ __launch_bounds__(FT, 4) void k_gemm_f32_ax(const void* const* __restrict__ ptrs, double* __restrict__ ws,
                                                      const GemmTask* __restrict__ tasks,
                                                      const TileRef* __restrict__ tiles, int ntiles, int N) {
    gemm_f32_body<0>(ptrs, ws, tasks, tiles, ntiles, N);
}
__global__ __launch_bounds__(FT) void k_gemm_f32_atx(const void* const* __restrict__ ptrs, double* __restrict__ ws,
                                                     const GemmTask* __restrict__ tasks,
                                                     const TileRef* __restrict__ tiles, int ntiles, int N) {
    gemm_f32_body<1>(ptrs, ws, tasks, tiles, ntiles, N);
}

hipError_t prepare_gemm_f32_launches() {
    static unsigned long long d0 = 0, d1 = 0;
    hipError_t e = set_lds_limit_once((const void*)k_gemm_f32_ax, (int)(sizeof(float) * (size_t)(2 * XSZ)), &d0);
    if (e == hipSuccess) e = set_lds_limit_once((const void*)k_gemm_f32_atx, (int)(sizeof(float) * (size_t)(2 * XSZ)), &d1);
    return e;
}

hipError_t launch_gemm_f32(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                           const TileRef* tiles, int ntiles, int N, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (N < 1 || N > FN) return hipErrorInvalidValue;
    const size_t lds = sizeof(float) * (size_t)(2 * XSZ);    // X's two slab buffers
    hipError_t e = prepare_gemm_f32_launches();
    if (e != hipSuccess) return e;
    dim3 g(ntiles), b(FT);
    if (op == 0) hipLaunchKernelGGL(k_gemm_f32_ax, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    else hipLaunchKernelGGL(k_gemm_f32_atx, g, b, lds, s, ptrs, ws, tasks, tiles, ntiles, N);
    return hipGetLastError();
}

}  // namespace hsvd
