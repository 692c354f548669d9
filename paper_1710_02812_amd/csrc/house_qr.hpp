// Register-resident Householder QR of a small block, shared by the tall-skinny
// QR kernels and the merge cores.
#pragma once
#include "device_common.hpp"

namespace hsvd {

// Register-resident Householder QR of one rows x w block (rows <= LANES * RMAX,
// w <= CPL * NTHR / LANES) with NTHR threads = NG groups of LANES lanes.  Column c
// lives in slot c / NG of group c % NG (CPL slots per group), row r in lane
// r % LANES (index r / LANES of the slot), so the trailing matrix never travels
// through LDS; per step only the pivot reflector is broadcast through LDS, and a
// lane reads each pivot value once for all of its slots.  Reflectors follow the
// dlarfg convention (H = I - tau v v^T, v_j = 1, R_jj = beta); with WITH_T the
// compact-WY factor T of Q = H_0 ... H_{w-1} = I - V T V^T is built alongside
// (dlarft forward/columnwise: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] z,
// z = V[:, 0:j]^T v_j).
//
// One barrier per step, with look-ahead: in step j every column c > j is updated
// with v_j, and the group of column j + 1, right after that column's update, forms
// v_{j+1} into the other half of a double buffer.  Columns c < j meanwhile form
// z_c = v_c^T v_j and, from the z of step j - 1, their row of T column j - 1 (each
// column owns one row of T, so T never needs a barrier of its own).
// KVMAX: pivot values kept in registers between the dot and the update when
// NT <= KVMAX (else read twice from LDS).
template <int LANES, int RMAX, bool WITH_T = true, int KVMAX = 8, int CPL = 1, int NTHR = 1024>
struct HouseQR {
    static constexpr int NG = NTHR / LANES;
    static constexpr int VB = LANES * RMAX;      // rows one column can hold
    static constexpr int WMAX = NG * CPL;        // columns the block can hold
    double x[CPL * RMAX];                        // slot s, register t: x[s * RMAX + t]

    // LDS doubles factor() needs: T (w x (w + 1)), tau (w), z (2w), two pivot buffers
    __host__ __device__ static constexpr size_t lds_doubles(int w) {
        return (size_t)w * (w + 1) + 3 * (size_t)w + 2 * (size_t)VB;
    }

    __device__ static double gsum(double v) { return LANES == 16 ? sum16(v) : sum8(v); }
    __device__ static int col_of(int s) { return (int)(threadIdx.x / LANES) + s * NG; }

    __device__ void load(const double* src, int64_t ld, int rows, int w) {
        const int gl = threadIdx.x % LANES;
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = col_of(s);
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                const int r = gl + LANES * t;
                x[s * RMAX + t] = (c < w && r < rows) ? src[(int64_t)c * ld + r] : 0.0;
            }
        }
    }

    // writes the factored block (R above/on the diagonal, reflectors below)
    __device__ void store(double* dst, int64_t ld, int rows, int w) const {
        const int gl = threadIdx.x % LANES;
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = col_of(s);
            if (c >= w) continue;
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                const int r = gl + LANES * t;
                if (r < rows) dst[(int64_t)c * ld + r] = x[s * RMAX + t];
            }
        }
    }

    // R (w x w, col-major ld w): upper triangle of the first min(rows, w) rows
    __device__ void store_r(double* R, int rows, int w) const {
        const int gl = threadIdx.x % LANES;
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = col_of(s);
            if (c >= w) continue;
#pragma unroll
            for (int t = 0; t < RMAX; ++t) {
                const int r = gl + LANES * t;
                if (r < w) R[(int64_t)c * w + r] = (r <= c && r < rows) ? x[s * RMAX + t] : 0.0;
            }
        }
    }

    // Squared norm of the rows r > j of slot s (registers t < NT; rows past the
    // block hold zeros).
    // Register TJ = j / LANES straddles row j; below it every register lies wholly above
    // row j, past it wholly below (the callers dispatch on the wave-uniform j / LANES,
    // so those registers need no per-lane test).
    template <int NT, int TJ>
    __device__ double norm_below_t(int s, int j) const {
        const int gl = threadIdx.x % LANES;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t < TJ) continue;
            const double m = (t > TJ || gl + LANES * t > j) ? x[s * RMAX + t] : 0.0;
            if (t & 1) s1 = fma(m, m, s1);
            else s0 = fma(m, m, s0);
        }
        return gsum(s0 + s1);
    }
    template <int NT>
    __device__ double norm_below(int s, int j) const {
        switch (j / LANES) {
#define HQ_NB(k) case k: if constexpr (k < NT) return norm_below_t<NT, k>(s, j); else break;
            HQ_NB(0) HQ_NB(1) HQ_NB(2) HQ_NB(3) HQ_NB(4) HQ_NB(5) HQ_NB(6) HQ_NB(7)
            HQ_NB(8) HQ_NB(9) HQ_NB(10) HQ_NB(11) HQ_NB(12) HQ_NB(13) HQ_NB(14) HQ_NB(15)
#undef HQ_NB
            default: break;
        }
        return 0.0;
    }

    // The scaled reflector into its registers and vb (zeros above row j, 1 at row j),
    // beta at row j; register TJ = j / LANES is the only one with a per-lane test.
    template <int NT, int TJ>
    __device__ void reflect_rows(int s, int j, double beta, double s2, double scal, double* vb) {
        const int gl = threadIdx.x % LANES;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int r = gl + LANES * t;
            double v = 0.0;
            if (t > TJ) {
                if (s2 > 0.0) x[s * RMAX + t] *= scal;
                v = x[s * RMAX + t];
            } else if (t == TJ) {
                if (r == j) { x[s * RMAX + t] = beta; v = 1.0; }
                else if (r > j) { if (s2 > 0.0) x[s * RMAX + t] *= scal; v = x[s * RMAX + t]; }
            }
            vb[r] = v;
        }
    }

    // Reflector of column j (slot s of the calling group): alpha = A_jj sits in
    // register j / LANES of the group's lane j % LANES, s2 is the squared norm below
    // the diagonal.  Leaves beta at row j and v below it in the registers, writes v_j
    // (0 above row j) into vb and tau_j into tau[j].  The square root and the
    // reciprocals come from the hardware estimates refined by Newton steps.
    template <int NT>
    __device__ void reflect(int s, int j, double s2, double* vb, double* tau) {
        const int gl = threadIdx.x % LANES;
        const int tj = j / LANES;
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (t == tj) a = x[s * RMAX + t];
        const int src = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & 63) - gl) + (j % LANES);
        const double alpha = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(a), src),
                                              __builtin_amdgcn_readlane(__double2loint(a), src));
        double beta = alpha, tau_j = 0.0, scal = 0.0;
        if (s2 > 0.0) {
            beta = -copysign(sqrt_nr(fma(alpha, alpha, s2)), alpha);
            tau_j = fma(-alpha, rcp_nr(beta), 1.0);           // (beta - alpha) / beta
            scal = rcp_nr(alpha - beta);                      // |alpha - beta| >= |beta| > 0
        }
        switch (tj) {
#define HQ_RF(k) case k: if constexpr (k < NT) reflect_rows<NT, k>(s, j, beta, s2, scal, vb); break;
            HQ_RF(0) HQ_RF(1) HQ_RF(2) HQ_RF(3) HQ_RF(4) HQ_RF(5) HQ_RF(6) HQ_RF(7)
            HQ_RF(8) HQ_RF(9) HQ_RF(10) HQ_RF(11) HQ_RF(12) HQ_RF(13) HQ_RF(14) HQ_RF(15)
#undef HQ_RF
            default: break;
        }
        if (gl == 0) tau[j] = tau_j;
    }

    // Row i of T column jj: -tau_jj sum_{l=i}^{jj-1} T[i][l] zz[l], by the group of row i.
    __device__ static void t_row(double* T, int ldt, int i, int jj, const double* zz, double tjj) {
        const int gl = threadIdx.x % LANES;
        double d = 0.0;
        for (int l = i + gl; l < jj; l += LANES) d = fma(T[(int64_t)l * ldt + i], zz[l], d);
        d = gsum(d);
        if (gl == 0) T[(int64_t)jj * ldt + i] = -tjj * d;
    }

    // lds scratch (lds_doubles(w)): T (w x (w+1)), tau (w), z (2w), vbuf (2 * VB);
    // T and z are unused without T.  Registers t >= NT must hold zeros and rows past
    // the block zeros (rows <= LANES * NT); loops run over the NT registers without
    // branches so that their LDS reads issue back to back.  All NTHR threads call
    // it; it ends on a barrier.
    template <int NT = RMAX>
    __device__ void factor(int rows, int w, double* T, double* tau, double* z, double* vbuf) {
        static_assert(NT >= 1 && NT <= RMAX, "NT out of range");
        constexpr bool CACHE = NT <= KVMAX;
        constexpr int KV = CACHE ? NT : 1;
        const int tid = threadIdx.x, nth = blockDim.x;
        const int grp = tid / LANES, gl = tid % LANES;
        const int kmax = rows < w ? rows : w;
        const int ldt = w + 1;
        if constexpr (WITH_T)
            for (int e = tid; e < w * ldt; e += nth) T[e] = 0.0;
        for (int j = kmax + tid; j < w; j += nth) tau[j] = 0.0;
        if (kmax > 0 && grp == 0) {                               // column 0: slot 0 of group 0
            const double s2 = norm_below<NT>(0, 0);
            reflect<NT>(0, 0, s2, vbuf, tau);
        }
        __syncthreads();
        if constexpr (CPL == 1) {
            // one column per group: the group of column c > j reads the pivot once,
            // forms the dot and updates; columns c < j form z (with T)
            for (int j = 0; j < kmax; ++j) {
                const double* vj = vbuf + (j & 1) * VB;
                const int c = grp;
                if (c < w && c > j) {
                    const double tj = tau[j];
                    if (tj != 0.0) {
                        double v[KV];
                        double d0 = 0.0, d1 = 0.0;
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            const double vt = vj[gl + LANES * t];             // broadcast reads
                            if (CACHE) v[t < KV ? t : 0] = vt;
                            if (t & 1) d1 = fma(vt, x[t], d1);
                            else d0 = fma(vt, x[t], d0);
                        }
                        const double f = tj * gsum(d0 + d1);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            x[t] = fma(-f, CACHE ? v[t < KV ? t : 0] : vj[gl + LANES * t], x[t]);
                    }
                    if (c == j + 1 && j + 1 < kmax) {                  // look-ahead reflector
                        const double s2 = norm_below<NT>(0, j + 1);
                        reflect<NT>(0, j + 1, s2, vbuf + ((j + 1) & 1) * VB, tau);
                    }
                } else if (WITH_T && c < j) {
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const double v = vj[gl + LANES * t];
                        if (t & 1) d1 = fma(v, x[t], d1);
                        else d0 = fma(v, x[t], d0);
                    }
                    const double d = gsum(d0 + d1);
                    if (gl == 0) z[(j & 1) * w + c] = d;              // z_c = v_c^T v_j
                    if (c < j - 1) t_row(T, ldt, c, j - 1, z + ((j - 1) & 1) * w, tau[j - 1]);
                    else if (gl == 0) T[(int64_t)(j - 1) * ldt + (j - 1)] = tau[j - 1];
                }
                __syncthreads();
            }
        } else {
            // A wave's lane groups share one instruction stream, so the step runs in
            // three phases: the updates of every column c > j (both slots), then the
            // look-ahead reflector of column j + 1 (the step's critical path), then z
            // and the T rows of the columns c < j.
            // the wave holding column j + 1 forms the next reflector, the step's critical
            // path: it runs at raised issue priority until the reflector is out, ahead of
            // the update work of the other waves on its SIMD
            const int my_wave = __builtin_amdgcn_readfirstlane(tid >> 6);
            for (int j = 0; j < kmax; ++j) {
                const bool lead = j + 1 < kmax && ((((j + 1) % NG) * LANES) >> 6) == my_wave;
                if (lead) __builtin_amdgcn_s_setprio(2);
                const double* vj = vbuf + (j & 1) * VB;
                const double tj = tau[j];
                // the group reads the pivot only if one of its columns updates or forms z
                bool need = false;
#pragma unroll
                for (int s = 0; s < CPL; ++s) {
                    const int c = grp + s * NG;
                    need = need || (c < w && ((c > j && tj != 0.0) || (WITH_T && c < j)));
                }
                double v[KV];
                if (CACHE && need) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) v[t < KV ? t : 0] = vj[gl + LANES * t];   // broadcast reads
                }
                auto dot_v = [&](int s) {
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const double vt = CACHE ? v[t < KV ? t : 0] : vj[gl + LANES * t];
                        if (t & 1) d1 = fma(vt, x[s * RMAX + t], d1);
                        else d0 = fma(vt, x[s * RMAX + t], d0);
                    }
                    return gsum(d0 + d1);
                };
#pragma unroll
                for (int s = 0; s < CPL; ++s) {                     // updates
                    const int c = grp + s * NG;
                    if (c < w && c > j && tj != 0.0) {
                        const double f = tj * dot_v(s);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            x[s * RMAX + t] = fma(-f, CACHE ? v[t < KV ? t : 0] : vj[gl + LANES * t],
                                                  x[s * RMAX + t]);
                    }
                }
#pragma unroll
                for (int s = 0; s < CPL; ++s) {                     // look-ahead reflector
                    const int c = grp + s * NG;
                    if (c == j + 1 && j + 1 < kmax) {
                        const double s2 = norm_below<NT>(s, j + 1);
                        reflect<NT>(s, j + 1, s2, vbuf + ((j + 1) & 1) * VB, tau);
                    }
                }
                if (lead) __builtin_amdgcn_s_setprio(0);
                if (WITH_T) {
#pragma unroll
                    for (int s = 0; s < CPL; ++s) {                 // z and T rows
                        const int c = grp + s * NG;
                        if (c < j) {
                            const double d = dot_v(s);
                            if (gl == 0) z[(j & 1) * w + c] = d;      // z_c = v_c^T v_j
                            if (c < j - 1) t_row(T, ldt, c, j - 1, z + ((j - 1) & 1) * w, tau[j - 1]);
                            else if (gl == 0) T[(int64_t)(j - 1) * ldt + (j - 1)] = tau[j - 1];
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (WITH_T && kmax > 0) {
            const int J = kmax - 1;
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = grp + s * NG;
                if (c < J) t_row(T, ldt, c, J, z + (J & 1) * w, tau[J]);
                else if (c == J && gl == 0) T[(int64_t)J * ldt + J] = tau[J];
            }
        }
        __syncthreads();
    }
};


}  // namespace hsvd
