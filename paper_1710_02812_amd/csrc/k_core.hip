// Small dense SVD cores by one-sided (Hestenes) Jacobi in float64.
//
// Each work-group owns one core matrix G (at most 128 x 128) resident in LDS:
//   CORE_UPPER   : G = R, the triangular factor of a panel QR;
//   CORE_UPPER_T : G = R^T;
//   CORE_MERGE   : G = E = [[S1, C S2], [0, R S2]] of one merge step (Section 3,
//                  eq. orthmerge1 with the lower-right block R S2), built compactly
//                  from the two children's active ranks r1, r2.
// Columns are orthogonalised pairwise: a sweep visits every pair once through a
// round-robin tournament, so each round rotates nc/2 disjoint pairs in parallel,
// one lane group per pair (dot product by shuffle reduction, rotation in LDS).
// A pair is rotated when |g_a . g_b| > tol * |g_a| |g_b|; sweeps stop after a sweep
// without rotations.  At convergence G = U S (V not needed for merges, which
// drop the right factors); the optional accumulated rotations give V.
// Columns are then sorted by norm, the truncation rule picks the rank r, and the
// normalised left vectors, singular values and (optionally) V are written.
#include "hsvd_internal.hpp"
#include "device_common.hpp"

namespace hsvd {

constexpr int CORE_THREADS = 1024;

__device__ int select_rank(const double* sig, int nc, const CoreTask& t, const int* iws, int nr) {
    if (nc == 0) return 0;
    const double s0 = sig[0];
    if (!(s0 > 0.0)) return 0;
    const int fr = t.floor_rows;
    const int fc = t.floor_cols < 0 ? nc : t.floor_cols;
    const double floor = (double)(fr > fc ? fr : fc) * kEps * s0;
    int nonzero = 0;
    while (nonzero < nc && sig[nonzero] > floor) ++nonzero;
    int r;
    if (t.fixed_rank_slot >= 0) {
        r = iws[t.fixed_rank_slot];
    } else if (t.rule == 0) {
        r = 0;
        while (r < nc && sig[r] >= t.tol * s0) ++r;
    } else {
        // smallest r whose discarded tail sum_{i>=r} s_i^2 is <= tol^2 * total,
        // tails accumulated from the smallest value up
        double total = 0.0;
        for (int i = nc - 1; i >= 0; --i) total += sig[i] * sig[i];
        const double lim = t.tol * t.tol * total;
        double tail = 0.0;
        r = nc;
        for (int i = nc - 1; i >= 0; --i) {
            tail += sig[i] * sig[i];
            if (tail <= lim) r = i;
            else break;
        }
    }
    if (r > nonzero) r = nonzero;
    if (r > t.kcap) r = t.kcap;
    (void)nr;
    return r;
}

__global__ __launch_bounds__(CORE_THREADS) void k_core(double* __restrict__ ws, int* __restrict__ iws,
                                                       const CoreTask* __restrict__ tasks,
                                                       int maxdim, int max_sweeps,
                                                       unsigned* __restrict__ flags, int with_v) {
    extern __shared__ double sm[];
    const CoreTask t = tasks[blockIdx.x];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane64 = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const int ldg = maxdim + 1;
    double* G = sm;
    double* V = G + (int64_t)maxdim * ldg;
    double* d = V + (with_v ? (int64_t)maxdim * ldg : 0);
    double* sig = d + maxdim + 1;
    int* perm = (int*)(sig + maxdim);
    __shared__ int s_nr, s_nc, s_r1, s_r2, s_rot, s_bad, s_rank;

    if (tid == 0) {
        int nr, nc, r1 = 0, r2 = 0;
        if (t.mode == CORE_MERGE) {
            r1 = iws[t.rank1];
            r2 = iws[t.rank2];
            nr = nc = r1 + r2;
        } else {
            nr = nc = (t.rank_in >= 0) ? iws[t.rank_in] : t.dim;
        }
        if (nc > maxdim) { nr = nc = maxdim; }
        s_nr = nr; s_nc = nc; s_r1 = r1; s_r2 = r2; s_bad = 0;
    }
    __syncthreads();
    const int nr = s_nr, nc = s_nc, r1 = s_r1;
    const bool accv = (t.v_off >= 0) && with_v;

    // ---- load the core
    int bad = 0;
    for (int e = tid; e < nr * nc; e += nth) {
        const int j = e / nr, i = e - j * nr;
        double v = 0.0;
        if (t.mode == CORE_UPPER) {
            v = (i <= j) ? ws[t.m_off + (int64_t)j * t.m_ld + i] : 0.0;
        } else if (t.mode == CORE_UPPER_T) {
            v = (j <= i) ? ws[t.m_off + (int64_t)i * t.m_ld + j] : 0.0;
        } else if (t.mode == CORE_DENSE) {
            v = ws[t.m_off + (int64_t)j * t.m_ld + i];
        } else {
            if (j < r1) {
                v = (i == j) ? ws[t.s1_off + j] : 0.0;
            } else {
                const int j2 = j - r1;
                const double s2 = ws[t.s2_off + j2];
                if (i < r1) v = ws[t.c_off + (int64_t)j2 * t.c_ld + i] * s2;
                else {
                    const int i2 = i - r1;
                    v = (i2 <= j2) ? ws[t.r_off + (int64_t)j2 * t.r_ld + i2] * s2 : 0.0;
                }
            }
        }
        if (!finite_d(v)) bad = 1;
        G[(int64_t)j * ldg + i] = v;
    }
    if (accv)
        for (int e = tid; e < nc * nc; e += nth) {
            const int j = e / nc, i = e - j * nc;
            V[(int64_t)j * ldg + i] = (i == j) ? 1.0 : 0.0;
        }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();

    // ---- one-sided Jacobi sweeps
    const int N = nc + (nc & 1);
    const int npairs = N >> 1;
    int gsz = 64;
    while (gsz > 1 && gsz * npairs > nth) gsz >>= 1;
    const int grp = tid / gsz, gl = tid - grp * gsz;
    const double tol = (double)(nr > 1 ? nr : 1) * kEps;
    bool converged = (nc <= 1) || s_bad;
    int sweep = 0;
    for (; sweep < max_sweeps && !converged; ++sweep) {
        for (int j = wave; j < nc; j += nw) {
            double s = 0.0;
            for (int i = lane64; i < nr; i += 64) {
                const double g = G[(int64_t)j * ldg + i];
                s = fma(g, g, s);
            }
            s = wave_sum(s);
            if (lane64 == 0) d[j] = s;
        }
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int round = 0; round < N - 1; ++round) {
            if (grp < npairs) {
                int a, b;
                if (grp == 0) { a = round; b = N - 1; }
                else { a = (round + grp) % (N - 1); b = (round + N - 1 - grp) % (N - 1); }
                const bool valid = (a < nc) && (b < nc);
                double c = 0.0;
                if (valid)
                    for (int i = gl; i < nr; i += gsz)
                        c = fma(G[(int64_t)a * ldg + i], G[(int64_t)b * ldg + i], c);
                c = group_sum(c, gsz);
                if (valid) {
                    const double da = d[a], db = d[b];
                    const double na = sqrt(da), nb = sqrt(db);
                    if (na > 0.0 && nb > 0.0 && fabs(c) > tol * na * nb) {
                        const double zeta = (db - da) / (2.0 * c);
                        const double az = fabs(zeta);
                        const double tt = (az > 1e150) ? 0.5 / zeta
                                                       : copysign(1.0 / (az + sqrt(1.0 + zeta * zeta)), zeta);
                        const double cs = 1.0 / sqrt(1.0 + tt * tt);
                        const double sn = cs * tt;
                        double* ga = G + (int64_t)a * ldg;
                        double* gb = G + (int64_t)b * ldg;
                        for (int i = gl; i < nr; i += gsz) {
                            const double x = ga[i], y = gb[i];
                            ga[i] = cs * x - sn * y;
                            gb[i] = sn * x + cs * y;
                        }
                        if (accv) {
                            double* va = V + (int64_t)a * ldg;
                            double* vb = V + (int64_t)b * ldg;
                            for (int i = gl; i < nc; i += gsz) {
                                const double x = va[i], y = vb[i];
                                va[i] = cs * x - sn * y;
                                vb[i] = sn * x + cs * y;
                            }
                        }
                        if (gl == 0) {
                            d[a] = da - tt * c;
                            d[b] = db + tt * c;
                            s_rot = 1;
                        }
                    }
                }
            }
            __syncthreads();
        }
        converged = (s_rot == 0);
        __syncthreads();
    }
    if (tid == 0 && flags) {
        unsigned f = 0;
        if (s_bad) f |= 1u;
        if (!converged) f |= 2u;
        if (f) atomicOr(flags, f);
    }

    // ---- singular values (exact column norms), sort descending
    for (int j = wave; j < nc; j += nw) {
        double s = 0.0;
        for (int i = lane64; i < nr; i += 64) {
            const double g = G[(int64_t)j * ldg + i];
            s = fma(g, g, s);
        }
        s = wave_sum(s);
        if (lane64 == 0) d[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < nc; j += nth) {
        const double sj = d[j];
        int pos = 0;
        for (int i = 0; i < nc; ++i) {
            const double si = d[i];
            pos += (si > sj) || (si == sj && i < j);
        }
        perm[pos] = j;
        sig[pos] = sj;
    }
    __syncthreads();
    if (tid == 0) {
        const int r = s_bad ? 0 : select_rank(sig, nc, t, iws, nr);
        s_rank = r;
        if (t.rank_out >= 0) iws[t.rank_out] = r;
    }
    __syncthreads();
    const int r = s_rank;

    // ---- outputs
    for (int i = tid; i < t.out_w; i += nth) ws[t.sig_off + i] = (i < r) ? sig[i] : 0.0;
    if (t.mode == CORE_MERGE) {
        const int rowsT = t.t_ld, rowsU = t.u_ld, r2 = s_r2;
        for (int e = tid; e < rowsT * t.out_w; e += nth) {
            const int i = e / rowsT, j = e - i * rowsT;
            ws[t.t_off + (int64_t)i * t.t_ld + j] =
                (i < r && j < r1) ? G[(int64_t)perm[i] * ldg + j] / sig[i] : 0.0;
        }
        for (int e = tid; e < rowsU * t.out_w; e += nth) {
            const int i = e / rowsU, j = e - i * rowsU;
            ws[t.u_off + (int64_t)i * t.u_ld + j] =
                (i < r && j < r2) ? G[(int64_t)perm[i] * ldg + r1 + j] / sig[i] : 0.0;
        }
    } else if (t.u_off >= 0) {
        const int rowsU = t.dim;
        for (int e = tid; e < rowsU * t.out_w; e += nth) {
            const int i = e / rowsU, j = e - i * rowsU;
            ws[t.u_off + (int64_t)i * t.u_ld + j] =
                (i < r && j < nr) ? G[(int64_t)perm[i] * ldg + j] / sig[i] : 0.0;
        }
    }
    if (accv) {
        const int rowsV = t.dim;
        for (int e = tid; e < rowsV * t.out_w; e += nth) {
            const int i = e / rowsV, j = e - i * rowsV;
            ws[t.v_off + (int64_t)i * t.v_ld + j] = (i < r && j < nc) ? V[(int64_t)perm[i] * ldg + j] : 0.0;
        }
    }
}

hipError_t launch_core(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                         int max_sweeps, unsigned* flags, int with_v, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * ((size_t)maxdim * (maxdim + 1) * (with_v ? 2 : 1) +
                                         2 * (size_t)maxdim + 1) + sizeof(int) * maxdim + 64;
    hipError_t e = hipFuncSetAttribute((const void*)k_core,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_core, dim3(ntasks), dim3(CORE_THREADS), lds, s, ws, iws, tasks, maxdim,
                       max_sweeps, flags, with_v);
    return hipGetLastError();
}

}  // namespace hsvd
