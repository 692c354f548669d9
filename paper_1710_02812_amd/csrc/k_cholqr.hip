// Cholesky QR passes: the fast path of the tall-skinny QR for well-conditioned panels
// (the merge complements, the slab re-projection and the projection, whose condition
// numbers are a few thousand), with the Householder TSQR as the fallback.
//
//   pass 1: G = P^T P,   R1 = chol(G),   M1 = R1^{-1}
//   (Q1 = P M1 by the thin product kernel)
//   pass 2: G2 = Q1^T Q1, R2 = chol(G2), R = R2 R1 -> the panel's R, M2 = R2^{-1}
//   (the apply then forms Q X = Q1 (M2 X) with thin products)
//
// Partial Grams of 256-row chunks run on the float64 matrix cores and are summed up a
// tree of fan-in 8 (the last child of a node to arrive adds its siblings, in child
// order); the work-group that completes the root factors the panel's Gram matrix.
// Fallback (flag 1: the Householder kernels run, these outputs are ignored): a pass-1
// pivot below 1e-10 of its column's squared norm (the column is nearly a combination
// of the previous ones), or ||Q1^T Q1 - I||_F > 1/4 over the live columns (a first pass
// that far from orthonormal would leave the second short of working precision).
// Exactly zero columns (zero padding past a rank) are dead: zero rows of R and zero
// columns of M, so that P = Q R and the singular values of R are those of P.
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

// Scratch of a panel (cq_size doubles from cq_off): R1 | M1 | M2 | chunk parts (nch w^2) |
// node sums | Q1 (h x w, ld h)

// Value of v in lane l (l uniform across the wave).
__device__ __forceinline__ double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 1 / p to within an ulp or so: the hardware estimate and two Newton steps.
__device__ __forceinline__ double recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// Steps JB .. JB + 15 of the elimination below (their columns are held by wave JB / 16).
// Every wave evaluates the pivot arithmetic (only the owner's is kept), so that one
// instruction stream interleaves it with the reads of row j; the owner uses its
// multipliers from registers, the others read them from Lm after the barrier.
template <int JB>
__device__ __forceinline__ void elim_steps(double (&x)[16], double& dpiv, bool& failed, int w, int q, int lane,
                                           double d0l, bool check, double* Lm) {
    const bool owner = q == JB / 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = JB + jj;
        if (j < w) {
            const double piv = readlane_d(x[jj], j);
            const double d0j = readlane_d(d0l, j);
            const bool live = d0j != 0.0;
            failed |= check && owner && live && !(piv > 1e-10 * d0j);
            const bool use = live && piv > 0.0;
            const double rp = use ? recip(piv) : 0.0;
            const double m = lane > j ? x[jj] * rp : 0.0;
            if (owner) Lm[j * 64 + lane] = m;
            dpiv = (owner && lane == j) ? (use ? piv : 0.0) : dpiv;
            const double xc = lane == j ? 1.0 : (lane > j ? -m : 0.0);   // column j of L^-1
            double row[16];                           // row j of this wave's columns
#pragma unroll
            for (int k = 0; k < 16; ++k) row[k] = readlane_d(x[k], j);
            __syncthreads();
            if (owner) {
#pragma unroll
                for (int k = 0; k < 16; ++k) x[k] = k == jj ? xc : fma(-m, row[k], x[k]);
            } else {
                const double mm = Lm[j * 64 + lane];
#pragma unroll
                for (int k = 0; k < 16; ++k) x[k] = fma(-mm, row[k], x[k]);
            }
        }
    }
}

// Cholesky factor and inverse of a w x w Gram matrix G (w <= 64, col-major, ld) by
// elimination without pivoting, on 256 threads: lane i holds row i, wave q columns
// 16 q .. 16 q + 15, in registers.  Step j subtracts m_ij = G(i, j) / G(j, j) times row
// j from each row i > j; with G = L D L^T (L unit lower, the multipliers; D the pivots)
// R = D^1/2 L^T.  After step j column j holds the column j of L^-1 that the same row
// operations build from the identity (a column of L^-1 starts at step j, just as column
// j of G ends).  Then M = L^-T D^-1/2 = R^-1; R and M come from the same L, so that
// M R = (L L^-1)^T is the identity to working precision (Q1 R1 = P M1 R1 = P), with no
// back substitution.  d0: G's diagonal (0 marks a dead column: its row of R and column
// of M stay zero).  With check, a live pivot at or below 1e-10 of its column's squared
// norm sets *fail.  Lm: 64 x 64 doubles of LDS for the multipliers (may be G's own
// storage).  Writes R (upper, ld ldr) and M (upper, ld ldm), zero below the diagonal.
__device__ __forceinline__ void chol_elim(const double* G, int ld, const double* d0, int w, bool check,
                                          double* Lm, double* dl, int* fail, double* R, int ldr, double* M,
                                          int ldm) {
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = 16 * q + k;
        x[k] = (lane < w && c < w) ? G[(int64_t)c * ld + lane] : 0.0;
    }
    const double d0l = lane < w ? d0[lane] : 0.0;
    __syncthreads();                                  // G read before Lm (over it) is written
    double dpiv = 0.0;
    bool failed = false;
    elim_steps<0>(x, dpiv, failed, w, q, lane, d0l, check, Lm);
    if (w > 16) elim_steps<16>(x, dpiv, failed, w, q, lane, d0l, check, Lm);
    if (w > 32) elim_steps<32>(x, dpiv, failed, w, q, lane, d0l, check, Lm);
    if (w > 48) elim_steps<48>(x, dpiv, failed, w, q, lane, d0l, check, Lm);
    if (lane >> 4 == q) dl[lane] = dpiv;              // pivots D (0: dead or failed)
    if (failed) *fail = 1;
    __syncthreads();
    // column `lane` of M: M(r, c) = L^-1(c, r) / sqrt(D_c) for r <= c
    if (lane < w) {
        const double dc = dl[lane];
        const double rs = dc > 0.0 ? 1.0 / sqrt(dc) : 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int r = 16 * q + k;
            if (r < w) M[(int64_t)lane * ldm + r] = r <= lane ? x[k] * rs : 0.0;
        }
    }
    // R(j, i) = sqrt(D_j) m_ij right of the diagonal
    for (int e = tid; e < w * w; e += blockDim.x) {
        const int i = e / w, j = e - i * w;
        const double sj = sqrt(dl[j]);
        R[(int64_t)i * ldr + j] = i > j ? sj * Lm[j * 64 + i] : (i == j ? sj : 0.0);
    }
    __syncthreads();
}

template <int PASS>
__global__ __launch_bounds__(256) void k_cholqr(double* __restrict__ ws, int* __restrict__ iws,
                                                const TsqrTask* __restrict__ tasks,
                                                const ChunkRef* __restrict__ chunks, int w, int ch) {
    __shared__ double As[mfma_lds_a<0>()];
    __shared__ double Bs[mfma_lds_b()];
    __shared__ double d0[64];
    __shared__ double s_d[64];
    __shared__ int s_last, s_fail, s_cfail;
    __shared__ double s_part[4];
    const ChunkRef cr = chunks[blockIdx.x];
    const TsqrTask t = tasks[cr.task];
    if (t.cq_flag < 0) return;
    if (PASS == 2 && iws[t.cq_flag] != 0) return;      // pass 1 already fell back
    const int tid = threadIdx.x;
    double* cq = ws + t.cq_off;
    double* R1 = cq;
    double* M1 = cq + (int64_t)w * w;
    double* M2 = cq + 2 * (int64_t)w * w;
    double* parts = cq + 3 * (int64_t)w * w;
    double* Q1 = cq + cq_q1(w, t.nch);
    const double* X = PASS == 1 ? ws + t.p_off : Q1;
    const int64_t ldx = PASS == 1 ? t.p_ld : t.h;
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    const int ww = w * w;
    // partial Gram X_c^T X_c (X_c^T is a row-major w x rows array)
    v4d acc[2][2];
    mfma_tile<double, 0>(X + row0, ldx, X + row0, ldx, w, w, rows, 0, 0, As, Bs, acc);
    double* part = parts + (int64_t)cr.chunk * ww;
    mfma_tile_out(w, w, 0, 0, acc, [&](int r, int c, double v) { part[(int64_t)c * w + r] = v; });
    // Sum up the tree: the last child of a node to arrive adds its (up to kCqFan)
    // siblings' sums in child order, all loads in flight at once; the root's sum is G.
    double* G = As;                                     // w x w, ld w + 1
    const int ld = w + 1;
    double* level = parts;                              // the current level's sums
    int n = t.nch, idx = cr.chunk, cnt = t.cq_cnt;
    for (;;) {
        const int parent = idx / kCqFan;
        const int first = parent * kCqFan, nchild = min(kCqFan, n - first);
        if (n > 1) {
            if (!tree_arrive(&iws[cnt + parent], nchild, &s_last)) return;
        } else {
            __syncthreads();
        }
        const int up = n > 1 ? cq_up(n) : 1;
        double* next = level + (int64_t)n * ww;
        double sum[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) sum[u] = 0.0;
#pragma unroll 2
        for (int c = 0; c < kCqFan; ++c) {
            const double* src = level + (int64_t)(first + min(c, nchild - 1)) * ww;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = min(tid + 256 * u, ww - 1);
                const double v = src[e];
                sum[u] += c < nchild ? v : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            if (e >= ww) continue;
            if (up == 1) {
                const int j = e / w, i = e - j * w;
                G[(int64_t)j * ld + i] = sum[u];
            } else {
                next[(int64_t)parent * ww + e] = sum[u];
            }
        }
        if (up == 1) break;
        level = next;
        cnt += up;
        n = up;
        idx = parent;
    }
    if (tid == 0) {
        s_fail = 0;
        s_cfail = 0;
    }
    __syncthreads();
    for (int j = tid; j < w; j += blockDim.x) d0[j] = G[(int64_t)j * ld + j];
    __syncthreads();
    if (PASS == 2) {
        // ||Q1^T Q1 - I||_F over the live columns, spread over the four waves
        double s = 0.0;
#pragma unroll 4
        for (int e = tid; e < w * w; e += 256) {
            const int j = e / w, i = e - j * w;
            const double v = G[(int64_t)j * ld + i] - (i == j ? 1.0 : 0.0);
            s = (d0[i] != 0.0 && d0[j] != 0.0) ? fma(v, v, s) : s;
        }
        s = wave_sum(s);
        if ((tid & 63) == 0) s_part[tid >> 6] = s;
        __syncthreads();
        if (tid == 0 && !((s_part[0] + s_part[1]) + (s_part[2] + s_part[3]) <= 1.0 / 16.0)) s_fail = 1;
        __syncthreads();
        if (s_fail) {
            if (tid == 0) iws[t.cq_flag] = 1;
            return;
        }
    }
    if (PASS == 1) {
        chol_elim(G, ld, d0, w, true, As, s_d, &s_cfail, R1, w, M1, w);
        if (tid == 0) iws[t.cq_flag] = s_cfail ? 1 : 0;
    } else {
        // R2 to LDS, M2 out; then the panel's R = R2 R1 (upper triangular)
        chol_elim(G, ld, d0, w, false, As, s_d, &s_cfail, Bs, w + 1, M2, w);
        for (int e = tid; e < w * w; e += blockDim.x) As[e] = R1[e];
        __syncthreads();
        double* Rout = ws + t.r_out;
        mfma_small(w, w, w, [&](int i, int l) { return Bs[(int64_t)l * (w + 1) + i]; },
                   [&](int l, int j) { return As[(int64_t)j * w + l]; },
                   [&](int i, int j, double v) { Rout[(int64_t)j * w + i] = i <= j ? v : 0.0; });
        if (tid == 0) iws[t.cq_flag] = 0;
    }
}

hipError_t launch_cholqr(int pass, double* ws, int* iws, const TsqrTask* tasks, const ChunkRef* chunks,
                         int nchunks, int w, int ch, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    if (w < 1 || w > 64 || ch > 256) return hipErrorInvalidValue;
    if (pass == 1)
        hipLaunchKernelGGL(k_cholqr<1>, dim3(nchunks), dim3(256), 0, s, ws, iws, tasks, chunks, w, ch);
    else
        hipLaunchKernelGGL(k_cholqr<2>, dim3(nchunks), dim3(256), 0, s, ws, iws, tasks, chunks, w, ch);
    return hipGetLastError();
}

}  // namespace hsvd
