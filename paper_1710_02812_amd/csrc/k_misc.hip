// Gaussian test matrices, fills, and the final sign-normalised output write.
#include "hsvd_internal.hpp"
#include "device_common.hpp"

namespace hsvd {

// Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit
// multiplies with the round constants and Weyl key increments published there.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// 53-bit uniform in the open interval (0, 1) from two 32-bit words.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

// out[e] ~ N(0, 1): Box-Muller on the Philox block of counter e/2 (rounded to T).
template <typename T>
__global__ void k_gaussian(T* out, int64_t count, uint64_t seed) {
    const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * pair >= count) return;
    const uint4 c = make_uint4((uint32_t)pair, (uint32_t)(pair >> 32), 0x5eedu, 0u);
    const uint2 k = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
    const uint4 x = philox4x32_10(c, k);
    const double u1 = u53(x.x, x.y), u2 = u53(x.z, x.w);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    out[2 * pair] = (T)(rad * cs);
    if (2 * pair + 1 < count) out[2 * pair + 1] = (T)(rad * sn);
}

__global__ void k_fill(double* p, int64_t count, double v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

// Column signs: flip so the largest-magnitude entry of u_j is positive (ties: lowest row).
// Matrix blockIdx.y of the batch, column blockIdx.x (blocks past its k return).
__global__ __launch_bounds__(256) void k_colsign(const double* __restrict__ ws, int* __restrict__ iws,
                                                 const OutputArgs* __restrict__ args) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const OutputArgs a = args[blockIdx.y];
    const int j = blockIdx.x;
    if (j >= a.k) return;
    const int r = iws[a.rank_slot];
    const double* u = ws + a.u_off + (int64_t)j * a.u_ld;
    double best = -1.0;
    int bi = 0x7fffffff;
    if (j < r)
        for (int i = threadIdx.x; i < a.m; i += blockDim.x) {
            const double v = fabs(u[i]);
            if (v > best) { best = v; bi = i; }       // first hit per thread is the lowest row
        }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o];
            const int i2 = si[threadIdx.x + o];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) iws[a.sign_off + j] = (j < r && si[0] < a.m && u[si[0]] < 0.0) ? -1 : 1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_write_u(const double* __restrict__ ws, const int* __restrict__ iws,
                                                 const OutputArgs* __restrict__ args,
                                                 void* const* __restrict__ ptrs) {
    __shared__ double tile[64][129];
    const OutputArgs a = args[blockIdx.y];
    T* __restrict__ U = (T*)ptrs[4 * blockIdx.y + 1];
    const int row0 = blockIdx.x * 64;
    if (row0 >= a.m) return;
    const int r = iws[a.rank_slot];
    const int rows = min(64, a.m - row0);
    for (int j0 = 0; j0 < a.k; j0 += 128) {
        const int cols = min(128, a.k - j0);
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * cols; e += blockDim.x) {
            const int jj = e / 64, i = e - jj * 64;
            const int j = j0 + jj;
            double v = 0.0;
            if (i < rows && j < r) v = iws[a.sign_off + j] * ws[a.u_off + (int64_t)j * a.u_ld + row0 + i];
            tile[i][jj] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
            const int i = e / cols, jj = e - i * cols;
            U[(int64_t)(row0 + i) * a.k + j0 + jj] = (T)tile[i][jj];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_write_v(const double* __restrict__ ws, const int* __restrict__ iws,
                                                 const OutputArgs* __restrict__ args,
                                                 void* const* __restrict__ ptrs) {
    const OutputArgs a = args[blockIdx.z];
    T* __restrict__ S = (T*)ptrs[4 * blockIdx.z + 2];
    T* __restrict__ Vt = (T*)ptrs[4 * blockIdx.z + 3];
    const int j = blockIdx.y;
    if (j >= a.k) return;
    const int r = iws[a.rank_slot];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double sg = (j < r) ? (double)iws[a.sign_off + j] : 0.0;
    if (c < a.n) Vt[(int64_t)j * a.n + c] = (T)(sg * ws[a.v_off + (int64_t)j * a.v_ld + c]);
    if (blockIdx.x == 0 && threadIdx.x == 0) S[j] = (T)((j < r) ? ws[a.sig_off + j] : 0.0);
}

hipError_t launch_gaussian(double* out, int64_t count, uint64_t seed, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t pairs = (count + 1) / 2;
    hipLaunchKernelGGL(k_gaussian<double>, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, out,
                       count, seed);
    return hipGetLastError();
}

hipError_t launch_gaussian_f32(float* out, int64_t count, uint64_t seed, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t pairs = (count + 1) / 2;
    hipLaunchKernelGGL(k_gaussian<float>, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, out,
                       count, seed);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

// Stopping test of Algorithm 2 (the relative change of the singular values between
// two iterations): one work-group, the items in turn, sums in a fixed order per lane
// and a fixed tree, so the decision does not depend on timing.
__global__ __launch_bounds__(256) void k_refine_check(const double* __restrict__ ws, int* __restrict__ iws,
                                                      const RefineCheck* __restrict__ items, int count,
                                                      double eps, int out_slot) {
    __shared__ double s_num[256], s_den[256];
    __shared__ int s_all;
    const int tid = threadIdx.x;
    if (tid == 0) s_all = 1;
    for (int i = 0; i < count; ++i) {
        const RefineCheck c = items[i];
        const int r = iws[c.rank_slot];
        double num = 0.0, den = 0.0;
        for (int j = tid; j < r; j += 256) {
            const double o = ws[c.sig_old + j], d = ws[c.sig_new + j] - o;
            num = fma(d, d, num);
            den = fma(o, o, den);
        }
        s_num[tid] = num;
        s_den[tid] = den;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) { s_num[tid] += s_num[tid + h]; s_den[tid] += s_den[tid + h]; }
            __syncthreads();
        }
        if (tid == 0 && !(s_num[0] <= eps * eps * s_den[0])) s_all = 0;
        __syncthreads();
    }
    if (tid == 0) iws[out_slot] = s_all;
}

hipError_t launch_refine_check(const double* ws, int* iws, const RefineCheck* items, int count, double eps,
                               int out_slot, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(256), 0, s, ws, iws, items, count, eps, out_slot);
    return hipGetLastError();
}

// Power-step convergence of the leaves (one work-group; one thread per item).  The
// leaf's truncation rank r follows the same rule as its core: a zero floor of
// max(rows, cols) eps s_0, then keep s_i >= tol s_0 (gamma) or the shortest prefix whose
// discarded energy is <= tol^2 of the total (Frobenius), at most kcap.
__global__ __launch_bounds__(256) void k_leaf_check(const double* __restrict__ ws, int* __restrict__ iws,
                                                    const LeafCheck* __restrict__ items, int count,
                                                    int step, int done_slot, const int* __restrict__ guard) {
    if (guard && *guard) return;
    __shared__ int s_all;
    if (threadIdx.x == 0) s_all = 1;
    __syncthreads();
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const LeafCheck c = items[i];
        const double* s = ws + c.sig_off;
        const double s0 = s[0];
        bool conv = true;
        if (s0 > 0.0) {
            const double floor = (double)(c.floor_rows > c.floor_cols ? c.floor_rows : c.floor_cols) * kEps * s0;
            int nz = 0;
            while (nz < c.w && s[nz] > floor) ++nz;
            int r;
            if (c.rule == 0) {
                r = 0;
                while (r < c.w && s[r] >= c.tol * s0) ++r;
            } else {
                double total = 0.0;
                for (int j = c.w - 1; j >= 0; --j) total += s[j] * s[j];
                const double lim = c.tol * c.tol * total;
                double tail = 0.0;
                r = c.w;
                for (int j = c.w - 1; j >= 0; --j) {
                    tail += s[j] * s[j];
                    if (tail <= lim) r = j;
                    else break;
                }
            }
            if (r > nz) r = nz;
            if (r > c.kcap) r = c.kcap;
            const double last = s[c.w - 1];
            if (r > 0 && last > floor && r < c.w) {
                const double rho = last / s[r - 1];
                double b = rho;
                for (int e = 0; e < 2 * step; ++e) b *= rho;      // rho^(2 step + 1)
                conv = b <= kLeafConvTol;
            }
        }
        if (!conv) atomicAnd(&s_all, 0);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_all) iws[done_slot] = 1;
}

hipError_t launch_leaf_check(const double* ws, int* iws, const LeafCheck* items, int count, int step,
                             int done_slot, const int* guard, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf_check, dim3(1), dim3(256), 0, s, ws, iws, items, count, step, done_slot, guard);
    return hipGetLastError();
}

__global__ void k_reset_state(unsigned* __restrict__ flags, int* __restrict__ iws,
                              const int* __restrict__ slots, int nslots) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) iws[slots[i]] = 0;
}

hipError_t launch_reset_state(unsigned* flags, int* iws, const int* slots, int nslots, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, flags, iws, slots, nslots);
    return hipGetLastError();
}

hipError_t launch_output(int fp32, const double* ws, int* iws, const OutputArgs* args, int count,
                         int kmax, int mmax, int nmax, void* const* ptrs, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsign, dim3(kmax, count), dim3(256), 0, s, ws, iws, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gu((mmax + 63) / 64, count), gv((nmax + 255) / 256, kmax, count);
    if (fp32) {
        hipLaunchKernelGGL(k_write_u<float>, gu, dim3(256), 0, s, ws, iws, args, ptrs);
        hipLaunchKernelGGL(k_write_v<float>, gv, dim3(256), 0, s, ws, iws, args, ptrs);
    } else {
        hipLaunchKernelGGL(k_write_u<double>, gu, dim3(256), 0, s, ws, iws, args, ptrs);
        hipLaunchKernelGGL(k_write_v<double>, gv, dim3(256), 0, s, ws, iws, args, ptrs);
    }
    return hipGetLastError();
}

}  // namespace hsvd
