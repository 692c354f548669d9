// Learned block rank: the features of a block's 16-column Gaussian sketch, and a
// 16-64-64-1 ReLU network (float16 weights, float32 arithmetic) that maps them to
// log2 of the rank the tolerance rule would keep, so that a leaf computes only the
// sketch columns it needs.  Training (forward, backward, Adam) runs in one
// persistent work-group; prediction takes one thread per block.
//
// Parameter vector (float32 master copy): W1 (64 x 16, row-major) | b1 (64) |
// W2 (64 x 64, row-major) | b2 (64) | w3 (64) | b3 (1).  The network always uses
// the weights rounded to float16 (the stored format); Adam updates the masters.
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include <hip/hip_fp16.h>

namespace hsvd {

constexpr int NI = 16, NH = 64, MB = kMlpBatch;
constexpr int O_W1 = 0, O_B1 = NH * NI, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH, O_W3 = O_B2 + NH,
              O_B3 = O_W3 + NH, NP = O_B3 + 1;
static_assert(NP == kMlpParams, "parameter layout");

__device__ __forceinline__ float half_round(float v) { return __half2float(__float2half_rn(v)); }

// steps > 0: `steps` Adam steps, minibatch of step s = samples (s0 + s) * MB + b mod
// count (b < MB), Adam step number t0 + s + 1; loss_out[s] = that step's loss.
// steps == 0: the gradient of minibatch s0 at the current weights into grad_out and
// its loss into loss_out[0]; nothing updated.
__global__ __launch_bounds__(256) void k_mlp_train(float* __restrict__ master, float* __restrict__ m1,
                                                   float* __restrict__ m2, const float* __restrict__ X,
                                                   const float* __restrict__ T, int count, int steps,
                                                   int s0, int t0, float lr, float* __restrict__ grad_out,
                                                   float* __restrict__ loss_out) {
    __shared__ float w[NP], g[NP];
    __shared__ float x[MB][NI], h1[MB][NH], h2[MB][NH], dz[MB][NH];
    __shared__ float dy[MB], tb[MB];
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int nsteps = steps > 0 ? steps : 1;
    for (int s = 0; s < nsteps; ++s) {
        const int sb = s0 + s;
        for (int i = tid; i < NP; i += 256) {
            w[i] = half_round(master[i]);
            g[i] = 0.0f;
        }
        for (int e = tid; e < MB * NI; e += 256) {
            const int b = e / NI, k = e - b * NI;
            const int idx = (int)(((int64_t)sb * MB + b) % count);
            x[b][k] = X[(int64_t)idx * NI + k];
        }
        if (tid < MB) tb[tid] = T[(int)(((int64_t)sb * MB + tid) % count)];
        __syncthreads();
        for (int e = tid; e < MB * NH; e += 256) {                 // layer 1
            const int b = e / NH, j = e - b * NH;
            float z = w[O_B1 + j];
#pragma unroll
            for (int k = 0; k < NI; ++k) z = fmaf(w[O_W1 + j * NI + k], x[b][k], z);
            h1[b][j] = fmaxf(z, 0.0f);
        }
        __syncthreads();
        for (int e = tid; e < MB * NH; e += 256) {                 // layer 2
            const int b = e / NH, j = e - b * NH;
            float z = w[O_B2 + j];
            for (int i = 0; i < NH; ++i) z = fmaf(w[O_W2 + j * NH + i], h1[b][i], z);
            h2[b][j] = fmaxf(z, 0.0f);
        }
        __syncthreads();
        float lpart = 0.0f;
        if (tid < MB) {                                            // output and loss
            float y = w[O_B3];
            for (int j = 0; j < NH; ++j) y = fmaf(w[O_W3 + j], h2[tid][j], y);
            const float r = y - tb[tid];
            dy[tid] = r / MB;
            lpart = 0.5f * r * r / MB;
        }
        // block sum of the loss (waves 0..3)
        float v = lpart;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0 && loss_out) loss_out[steps > 0 ? s : 0] = red[0] + red[1] + red[2] + red[3];
        if (tid < NH) {                                            // w3, b3
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a = fmaf(dy[b], h2[b][tid], a);
            g[O_W3 + tid] = a;
        } else if (tid == NH) {
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a += dy[b];
            g[O_B3] = a;
        }
        for (int e = tid; e < MB * NH; e += 256) {                 // dz2
            const int b = e / NH, j = e - b * NH;
            dz[b][j] = h2[b][j] > 0.0f ? dy[b] * w[O_W3 + j] : 0.0f;
        }
        __syncthreads();
        for (int e = tid; e < NH * NH; e += 256) {                 // W2
            const int j = e / NH, i = e - j * NH;
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a = fmaf(dz[b][j], h1[b][i], a);
            g[O_W2 + e] = a;
        }
        if (tid < NH) {                                            // b2
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a += dz[b][tid];
            g[O_B2 + tid] = a;
        }
        for (int e = tid; e < MB * NH; e += 256) {                 // dz1 (into h2)
            const int b = e / NH, i = e - b * NH;
            float a = 0.0f;
            for (int j = 0; j < NH; ++j) a = fmaf(dz[b][j], w[O_W2 + j * NH + i], a);
            h2[b][i] = h1[b][i] > 0.0f ? a : 0.0f;
        }
        __syncthreads();
        for (int e = tid; e < NH * NI; e += 256) {                 // W1
            const int j = e / NI, k = e - j * NI;
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a = fmaf(h2[b][j], x[b][k], a);
            g[O_W1 + e] = a;
        }
        if (tid < NH) {                                            // b1
            float a = 0.0f;
            for (int b = 0; b < MB; ++b) a += h2[b][tid];
            g[O_B1 + tid] = a;
        }
        __syncthreads();
        if (steps == 0) {
            for (int i = tid; i < NP; i += 256) grad_out[i] = g[i];
            return;
        }
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const int t = t0 + s + 1;
        const float c1 = 1.0f / (1.0f - powf(b1, (float)t)), c2 = 1.0f / (1.0f - powf(b2, (float)t));
        for (int i = tid; i < NP; i += 256) {
            const float gi = g[i];
            const float a = b1 * m1[i] + (1.0f - b1) * gi;
            const float bb = b2 * m2[i] + (1.0f - b2) * gi * gi;
            m1[i] = a;
            m2[i] = bb;
            master[i] -= lr * (a * c1) / (sqrtf(bb * c2) + eps);
        }
        __syncthreads();
    }
}

// One thread per sample: out[i] = network(X[i]) with float16-rounded weights.
__global__ __launch_bounds__(256) void k_mlp_predict(const float* __restrict__ master,
                                                     const float* __restrict__ X, int count,
                                                     float* __restrict__ out) {
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = half_round(master[i]);
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    float x[NI], a1[NH];
#pragma unroll
    for (int k = 0; k < NI; ++k) x[k] = X[(int64_t)s * NI + k];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float z = w[O_B1 + j];
#pragma unroll
        for (int k = 0; k < NI; ++k) z = fmaf(w[O_W1 + j * NI + k], x[k], z);
        a1[j] = fmaxf(z, 0.0f);
    }
    float y = w[O_B3];
    for (int j = 0; j < NH; ++j) {
        float z = w[O_B2 + j];
#pragma unroll
        for (int i = 0; i < NH; ++i) z = fmaf(w[O_W2 + j * NH + i], a1[i], z);
        y = fmaf(w[O_W3 + j], fmaxf(z, 0.0f), y);
    }
    out[s] = y;
}

// Squared Frobenius norm of each block (one work-group per GemmTask block).
// Energy ||A_b||_F^2 of every block, one 512-thread work-group per block.  The block is
// read as a flat sequence of 16-byte vectors (4 floats or 2 doubles of one row) when its
// rows allow it (and it has fewer than 2^31 of them), each thread keeping 8 in flight;
// otherwise element by element.
// Sums in float64, wave sums then one value per wave combined in wave order.
constexpr int EN_THREADS = 512;
constexpr int EN_UNROLL = 8;

template <typename T, typename V, int PER>
__device__ __forceinline__ double energy_vec(const T* base, int64_t lda, int rows, int cols) {
    const int nv = cols / PER;                    // vectors per row
    const int total = rows * nv;
    double s = 0.0;
    for (int e0 = threadIdx.x; e0 < total; e0 += EN_THREADS * EN_UNROLL) {
        V v[EN_UNROLL];
#pragma unroll
        for (int u = 0; u < EN_UNROLL; ++u) {
            const int e = e0 + u * EN_THREADS;
            if (e < total) {
                const int r = e / nv, c = e - r * nv;
                v[u] = *(const V*)(base + (int64_t)r * lda + (int64_t)c * PER);
            } else {
                v[u] = V{};
            }
        }
#pragma unroll
        for (int u = 0; u < EN_UNROLL; ++u)
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const double x = (double)v[u][q];
                s = fma(x, x, s);
            }
    }
    return s;
}

template <typename T>
__device__ __forceinline__ double energy_plain(const T* base, int64_t lda, int rows, int cols) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r)
        for (int c = threadIdx.x; c < cols; c += EN_THREADS) {
            const double x = (double)base[(int64_t)r * lda + c];
            s = fma(x, x, s);
        }
    return s;
}

__global__ __launch_bounds__(EN_THREADS) void k_block_energy(const void* const* __restrict__ ptrs, int fp32,
                                                             const GemmTask* __restrict__ tasks,
                                                             double* __restrict__ ws, int64_t out_off) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef double d2 __attribute__((ext_vector_type(2)));
    __shared__ double red[EN_THREADS / 64];
    const GemmTask t = tasks[blockIdx.x];
    double s;
    if (fp32) {
        const float* base = (const float*)ptrs[4 * t.mat] + t.a_off;
        const bool vec = t.cols % 4 == 0 && t.lda % 4 == 0 && ((uintptr_t)base & 15) == 0 &&
                         (int64_t)t.rows * (t.cols / 4) < ((int64_t)1 << 31) - EN_THREADS * EN_UNROLL;
        s = vec ? energy_vec<float, f4, 4>(base, t.lda, t.rows, t.cols) : energy_plain(base, t.lda, t.rows, t.cols);
    } else {
        const double* base = (const double*)ptrs[4 * t.mat] + t.a_off;
        const bool vec = t.cols % 2 == 0 && t.lda % 2 == 0 && ((uintptr_t)base & 15) == 0 &&
                         (int64_t)t.rows * (t.cols / 2) < ((int64_t)1 << 31) - EN_THREADS * EN_UNROLL;
        s = vec ? energy_vec<double, d2, 2>(base, t.lda, t.rows, t.cols) : energy_plain(base, t.lda, t.rows, t.cols);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < EN_THREADS / 64; ++w) tot += red[w];
        ws[out_off + blockIdx.x] = tot;
    }
}

// Features of block b from its sketch singular values (sig_off + 16 b, descending,
// zero padded) and energy: f_j = max(log10(s_{j+1}/s_1), -16) for j < 15,
// f_15 = log10(16 E / sum s^2); an all-zero block gives zeros.
__global__ void k_block_features(const double* __restrict__ ws, int64_t sig_off, int64_t energy_off,
                                 int nblocks, float* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    const double* s = ws + sig_off + 16 * (int64_t)b;
    const double E = ws[energy_off + b];
    float* f = out + 16 * (int64_t)b;
    if (!(s[0] > 0.0) || !(E > 0.0)) {
        for (int j = 0; j < 16; ++j) f[j] = 0.0f;
        return;
    }
    double ss = 0.0;
    for (int j = 0; j < 16; ++j) ss = fma(s[j], s[j], ss);
    for (int j = 0; j < 15; ++j) f[j] = (float)fmax(s[j + 1] > 0.0 ? log10(s[j + 1] / s[0]) : -16.0, -16.0);
    f[15] = (float)log10(E * 16.0 / ss);
}

hipError_t launch_mlp_train(float* master, float* m1, float* m2, const float* X, const float* T,
                            int count, int steps, int s0, int t0, float lr, float* grad_out,
                            float* loss_out, hipStream_t s) {
    if (count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(256), 0, s, master, m1, m2, X, T, count, steps, s0, t0,
                       lr, grad_out, loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const float* master, const float* X, int count, float* out, hipStream_t s) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_predict, dim3((count + 255) / 256), dim3(256), 0, s, master, X, count, out);
    return hipGetLastError();
}

hipError_t launch_block_energy(const void* const* ptrs, int fp32, const GemmTask* tasks, int ntasks,
                               double* ws, int64_t out_off, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_energy, dim3(ntasks), dim3(EN_THREADS), 0, s, ptrs, fp32, tasks, ws, out_off);
    return hipGetLastError();
}

__global__ void k_energy_sum(double* __restrict__ ws, int64_t part_off, const EnergySum* __restrict__ tasks,
                             int ntasks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntasks) return;
    const EnergySum t = tasks[i];
    const double* p = ws + part_off + t.first;
    double s = 0.0;
    for (int c = 0; c < t.count; ++c) s += p[c];
    ws[t.out] = s;
}

hipError_t launch_energy_sum(double* ws, int64_t part_off, const EnergySum* tasks, int ntasks, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_energy_sum, dim3((ntasks + 127) / 128), dim3(128), 0, s, ws, part_off, tasks, ntasks);
    return hipGetLastError();
}

hipError_t launch_block_features(const double* ws, int64_t sig_off, int64_t energy_off, int nblocks,
                                 float* out, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_features, dim3((nblocks + 127) / 128), dim3(128), 0, s, ws, sig_off,
                       energy_off, nblocks, out);
    return hipGetLastError();
}

}  // namespace hsvd
