// Register-resident Householder QR of a small block, shared by the tall-skinny
// QR kernels and the merge cores.
#pragma once
#include "device_common.hpp"

namespace hsvd {

// Register-resident Householder QR of one rows x w block (rows <= LANES * RMAX,
// w <= 1024 / LANES) with 1024 threads = groups of LANES lanes.  Column c lives in
// the registers of group c, row r in lane r % LANES (index r / LANES), so the
// trailing matrix never travels through LDS; per step only the pivot reflector is
// broadcast through LDS.
//
// Step j, phase 1: the owner of column j takes alpha = A_jj and the below-diagonal
// norm (left in LDS by step j-1), forms beta, tau_j and v_j (dlarfg convention:
// H = I - tau v v^T, v_j = 1, R_jj = beta) and publishes v_j; meanwhile the other
// groups finish column j-1 of the compact-WY factor T (dlarft forward/columnwise:
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] z with z = V[:, 0:j]^T v_j).
// Phase 2: every other column c forms v_j^T a_c; c > j is updated (c = j + 1 also
// leaves its next norm), c < j yields z_c.  Two barriers per step.  Without T
// (WITH_T = false) only R and the reflectors are produced: columns left of the
// pivot sit idle and T, z are not touched.
template <int LANES, int RMAX, bool WITH_T = true>
struct HouseQR {
    static constexpr int NG = 1024 / LANES;
    double x[RMAX];

    __device__ static double gsum(double v) { return LANES == 16 ? sum16(v) : sum8(v); }

    __device__ void load(const double* src, int64_t ld, int rows, int w) {
        const int c = threadIdx.x / LANES, gl = threadIdx.x % LANES;
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
            const int r = gl + LANES * t;
            x[t] = (c < w && r < rows) ? src[(int64_t)c * ld + r] : 0.0;
        }
    }

    // writes the factored block (R above/on the diagonal, reflectors below)
    __device__ void store(double* dst, int64_t ld, int rows, int w) const {
        const int c = threadIdx.x / LANES, gl = threadIdx.x % LANES;
        if (c >= w) return;
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
            const int r = gl + LANES * t;
            if (r < rows) dst[(int64_t)c * ld + r] = x[t];
        }
    }

    // R (w x w, col-major ld w): upper triangle of the first min(rows, w) rows
    __device__ void store_r(double* R, int rows, int w) const {
        const int c = threadIdx.x / LANES, gl = threadIdx.x % LANES;
        if (c >= w) return;
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
            const int r = gl + LANES * t;
            if (r < w) R[(int64_t)c * w + r] = (r <= c && r < rows) ? x[t] : 0.0;
        }
    }

    // T column j (rows i < j from z in ztmp; T_jj = tau_j).  The calling groups
    // number themselves vg = 0..ng-1 and stride over the rows.
    __device__ static void t_column(double* T, int ldt, int j, const double* ztmp, double tj,
                                    int vg, int ng) {
        const int gl = threadIdx.x % LANES;
        for (int i = vg; i < j; i += ng) {
            double d = 0.0;
            for (int l = i + gl; l < j; l += LANES) d = fma(T[(int64_t)l * ldt + i], ztmp[l], d);
            d = gsum(d);
            if (gl == 0) T[(int64_t)j * ldt + i] = -tj * d;
        }
        if (vg == 0 && gl == 0) T[(int64_t)j * ldt + j] = tj;
    }

    // lds scratch: T (w x (w+1)), tau (w), nrm (w), z (2w), vbuf (LANES * RMAX);
    // T and z are unused without T
    __device__ void factor(int rows, int w, double* T, double* tau, double* nrm, double* z,
                           double* vbuf) {
        const int tid = threadIdx.x, nth = blockDim.x;
        const int grp = tid / LANES, gl = tid % LANES;
        const int kmax = rows < w ? rows : w;
        const int ldt = w + 1;
        if constexpr (WITH_T)
            for (int e = tid; e < w * ldt; e += nth) T[e] = 0.0;
        if (grp == 0) {                                // norm of column 0 below the diagonal
            double s2 = 0.0;
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                const int r = gl + LANES * t;
                if (r > 0) s2 = fma(x[t], x[t], s2);
            }
            s2 = gsum(s2);
            if (gl == 0) nrm[0] = s2;
        }
        __syncthreads();
        for (int j = 0; j < kmax; ++j) {
            const int og = j;
            // ---- phase 1
            if (grp == og) {
                double a = 0.0;
#pragma unroll
                for (int t = 0; t < RMAX; ++t)
                    if (gl + LANES * t == j) a = x[t];
                const double alpha = gsum(a);
                const double sq = nrm[j];
                double beta = alpha, tj = 0.0, scal = 0.0;
                if (sq > 0.0) {
                    beta = -copysign(sqrt(alpha * alpha + sq), alpha);
                    tj = (beta - alpha) / beta;
                    scal = 1.0 / (alpha - beta);
                }
#pragma unroll
                for (int t = 0; t < RMAX; ++t) {
                    const int r = gl + LANES * t;
                    double v = 0.0;
                    if (r == j) { x[t] = beta; v = 1.0; }
                    else if (r > j) { if (sq > 0.0) x[t] *= scal; v = x[t]; }
                    vbuf[r] = v;                       // zero above row j and past the rows
                }
                if (gl == 0) tau[j] = tj;
            } else if (WITH_T && j > 0) {              // the other groups, renumbered
                t_column(T, ldt, j - 1, z + ((j - 1) & 1) * w, tau[j - 1], grp < og ? grp : grp - 1, NG - 1);
            }
            __syncthreads();
            // ---- phase 2
            const double tj = tau[j];
            double* zj = z + (j & 1) * w;
            const int c = grp;
            if (c < w && (WITH_T ? c != j : c > j)) {
                if (tj == 0.0) {
                    if (c == j + 1) {
                        double s2 = 0.0;
#pragma unroll
                        for (int t = 0; t < RMAX; ++t) {
                            const int r = gl + LANES * t;
                            if (r > j + 1 && r < rows) s2 = fma(x[t], x[t], s2);
                        }
                        s2 = gsum(s2);
                        if (gl == 0) nrm[j + 1] = s2;
                    }
                    if (WITH_T && c < j && gl == 0) zj[c] = 0.0;
                } else {
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int t = 0; t < RMAX; ++t) {
                        const double v = vbuf[gl + LANES * t];   // broadcast read within the wave
                        if (t & 1) d1 = fma(v, x[t], d1);
                        else d0 = fma(v, x[t], d0);
                    }
                    const double d = gsum(d0 + d1);
                    if (c < j) {
                        if (WITH_T && gl == 0) zj[c] = d;
                    } else {
                        const double f = tj * d;
                        double s2 = 0.0;
#pragma unroll
                        for (int t = 0; t < RMAX; ++t) {
                            const int r = gl + LANES * t;
                            x[t] = fma(-f, vbuf[r], x[t]);
                            const double m = (r > j + 1) ? x[t] : 0.0;
                            s2 = fma(m, m, s2);
                        }
                        if (c == j + 1) {
                            s2 = gsum(s2);
                            if (gl == 0) nrm[j + 1] = s2;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (WITH_T && kmax > 0)
            t_column(T, ldt, kmax - 1, z + ((kmax - 1) & 1) * w, tau[kmax - 1], grp, NG);
        for (int j = kmax + tid; j < w; j += nth) tau[j] = 0.0;
        __syncthreads();
    }
};


}  // namespace hsvd
