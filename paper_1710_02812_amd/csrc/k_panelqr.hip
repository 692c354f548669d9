// Tall-skinny QR of the leaves' sketch and power-step panels by repeated Cholesky QR,
// one work-group per panel (h x w, w <= kPanelQrMaxW), the whole factorization in
// one launch:
//
//   pass 1: G = P^T P + s I,  s = 11 (h w + w (w + 1)) u trace(P^T P),
//           R_1 = chol(G),   Q = P R_1^-1
//   pass p: G = Q^T Q,        R_p = chol(G),   Q <- Q R_p^-1
// and R = R_p ... R_1, so that P = Q R.  The shift keeps the first pass defined for
// any panel whose condition number is below about 1e13 and leaves Q within a
// condition number of about 1e5 (shifted Cholesky QR; Fukaya, Kannan, Nakatsukasa,
// Yamamoto and Yanagisawa, 2020); every later pass squares Q's distance from
// orthonormality.  The passes stop after the first pass p >= 2 whose Cholesky pivots,
// relative to the squared column norms of its input, are all >= 1/4 (that input was
// within a condition number of 2 of orthonormal, so the output is orthonormal to
// working precision); at most kPanelQrMaxPass passes.  A pass p >= 2 with a pivot at or
// below 1e-14 of its column's squared norm (a panel numerically rank deficient beyond
// what the shift covers, such as the sketch of an exactly low-rank block), a
// non-finite value, or the pass cap sets the panel's fallback flag: the Householder
// kernels then factor it and these outputs are ignored.  Exactly zero columns are
// dead: zero rows of R and zero columns of Q.  In the span-only mode the factorization
// stops after pass 1: Q = P R_1^-1 spans the panel and is well conditioned but not
// orthonormal to working precision, which is all a sketch's basis needs before the
// next power step.
//
// Products run on the float64 matrix cores (v_mfma_f64_16x16x4_f64) from slabs of 64
// rows staged through LDS (the next slab loaded into registers while the current one
// is multiplied): the Gram matrix as its upper-triangle 16 x 16 tiles, the
// product Q = X M (M = R_p^-1, upper triangular) as 64 x 16 tiles that stop at M's
// diagonal.  The Cholesky factor comes from elimination without pivoting with one row
// of G per lane (two halves of 64 rows) and 16 columns per wave held in registers: the
// same row operations turn the identity into L^-1 (G = L D L^T, R = D^1/2 L^T,
// M = L^-T D^-1/2), so that M R is the identity to working precision.
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

namespace {

constexpr int PQ_THREADS = 512;
constexpr int PQ_RS = 64;                    // rows per staged slab
constexpr int PQ_SP = PQ_RS + 1;             // LDS pitch of a staged column
constexpr int PQ_GP = kPanelQrMaxW + 1;      // LDS pitch of G / multipliers / M columns
constexpr int PQ_LDS_G = kPanelQrMaxW * PQ_GP;
constexpr int PQ_LDS_S = kPanelQrMaxW * PQ_SP;
constexpr size_t PQ_LDS_BYTES = sizeof(double) * (PQ_LDS_G + PQ_LDS_S + 2 * 128) + 64;

__device__ __forceinline__ double pq_readlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double pq_recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// Slab [row0, row0 + 64) of the panel X (col-major, ld), zero past h rows and past w
// columns (up to T * 16 columns): element e = tid + PQ_THREADS u (column e / 64, row
// e % 64) into v[u], then into S[c * PQ_SP + r].  Loading the next slab into registers
// before the current one's products keeps its latency off the slab loop.
constexpr int PQ_PF = kPanelQrMaxW / 16 * 2;   // slab elements per thread (T <= 6)
__device__ __forceinline__ void pq_load(const double* __restrict__ X, int64_t ld, int h, int w, int T,
                                        int row0, double (&v)[PQ_PF]) {
#pragma unroll
    for (int u = 0; u < PQ_PF; ++u) {
        const int e = threadIdx.x + PQ_THREADS * u;
        const int c = e >> 6, gr = row0 + (e & 63);
        v[u] = (u < 2 * T && c < w && gr < h) ? X[(int64_t)c * ld + gr] : 0.0;
    }
}
__device__ __forceinline__ void pq_put(const double (&v)[PQ_PF], int T, double* S) {
#pragma unroll
    for (int u = 0; u < PQ_PF; ++u) {
        const int e = threadIdx.x + PQ_THREADS * u;
        if (u < 2 * T) S[(e >> 6) * PQ_SP + (e & 63)] = v[u];
    }
}

// Elimination steps JB .. JB + 15 (columns of wave JB / 16).  x[h][k]: row lane + 64 h,
// column 16 q + k of the working matrix.  Every wave evaluates the pivot arithmetic
// (only the owner's is kept); the owner takes its multipliers from registers, the
// others read them from Lm after the barrier.
template <int JB>
__device__ __forceinline__ void pq_steps(double (&x)[2][16], double (&dpiv)[2], bool& failed, double& rho,
                                         int w, int q, int lane, const double (&d0l)[2], double thresh,
                                         double* Lm) {
    constexpr int H = JB / 64;
    const bool owner = q == JB / 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = JB + jj;
        if (j < w) {
            const int lj = (JB & 63) + jj;
            const double piv = pq_readlane(x[H][jj], lj);
            const double d0j = pq_readlane(d0l[H], lj);
            const bool live = d0j > 0.0;
            if (owner && live) {
                failed |= !(piv > thresh * d0j) || !finite_d(piv);
                rho = fmin(rho, piv / d0j);
            }
            const bool use = live && piv > 0.0;
            const double rp = use ? pq_recip(piv) : 0.0;
            double m0 = lane > j ? x[0][jj] * rp : 0.0;
            double m1 = lane + 64 > j ? x[1][jj] * rp : 0.0;
            if (owner) {
                Lm[j * PQ_GP + lane] = m0;
                if (lane + 64 < w) Lm[j * PQ_GP + lane + 64] = m1;
            }
            if (owner && lane == lj) dpiv[H] = use ? piv : 0.0;
            double row[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) row[k] = pq_readlane(x[H][k], lj);
            __syncthreads();
            if (!owner) {
                m0 = Lm[j * PQ_GP + lane];
                m1 = lane + 64 < w ? Lm[j * PQ_GP + lane + 64] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                x[0][k] = fma(-m0, row[k], x[0][k]);
                x[1][k] = fma(-m1, row[k], x[1][k]);
            }
            if (owner) {             // column j of L^-1 starts here
                x[0][jj] = lane == j ? 1.0 : (lane > j ? -m0 : 0.0);
                x[1][jj] = lane + 64 == j ? 1.0 : (lane + 64 > j ? -m1 : 0.0);
            }
        }
    }
}

}  // namespace

__global__ __launch_bounds__(PQ_THREADS) void k_panel_qr(double* __restrict__ ws, int* __restrict__ iws,
                                                         const TsqrTask* __restrict__ tasks, int w, int need_r,
                                                         const int* __restrict__ guard,
                                                         const int* __restrict__ order) {
    if (guard && *guard) return;                  // a skipped stage (every group returns)
    extern __shared__ double pq_sm[];
    double* Ga = pq_sm;                           // G, then the multipliers, then M
    double* Sb = Ga + PQ_LDS_G;                   // staged slab
    double* dl = Sb + PQ_LDS_S;                   // pivots D
    double* d0 = dl + 128;                        // G's diagonal (unshifted)
    __shared__ int s_fail;
    __shared__ double s_rho[8];
    __shared__ double s_tr[8];
    // panels in the launch's dispatch order (tallest first: the longest work-groups start
    // first and the launch's tail is short), or in task order
    const TsqrTask t = tasks[order ? order[blockIdx.x] : (int)blockIdx.x];
    if (t.pq_q_off < 0) return;
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int h = t.h;
    const int T = (w + 15) >> 4;                  // 16-column tiles
    const int K4 = (w + 3) & ~3;                  // reduction length of the products
    const int NT = T * (T + 1) / 2;               // upper-triangle Gram tiles
    const double* P = ws + t.p_off;
    double* Qd = ws + t.pq_q_off;
    const int64_t qld = t.pq_q_ld;
    double* Tbuf = ws + t.pq_scr;                 // R accumulation (2 w^2, ping-pong)
    bool failed_all = false;
    for (int pass = 1; pass <= kPanelQrMaxPass; ++pass) {
        const double* X = pass == 1 ? P : Qd;
        const int64_t ldx = pass == 1 ? t.p_ld : qld;
        // ---- Gram matrix: upper-triangle tiles, up to 3 per wave
        v4d acc[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
        int ti[3], tj[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            int tt = q + 8 * u, a = 0;
            if (tt >= NT) tt = 0;
            while (tt >= T - a) { tt -= T - a; ++a; }
            ti[u] = a;
            tj[u] = a + tt;
        }
        double pf[PQ_PF];
        pq_load(X, ldx, h, w, T, 0, pf);
        for (int row0 = 0; row0 < h; row0 += PQ_RS) {
            pq_put(pf, T, Sb);
            __syncthreads();
            if (row0 + PQ_RS < h) pq_load(X, ldx, h, w, T, row0 + PQ_RS, pf);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                if (q + 8 * u < NT) {
                    const double* sa = Sb + (ti[u] * 16 + li) * PQ_SP + lk;
                    const double* sbp = Sb + (tj[u] * 16 + li) * PQ_SP + lk;
#pragma unroll 4
                    for (int k0 = 0; k0 < PQ_RS; k0 += 4)
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[k0], sbp[k0], acc[u], 0, 0, 0);
                }
            }
            __syncthreads();
        }
        // G to LDS (both triangles), zero past w
        for (int e = tid; e < T * 16 * PQ_GP; e += PQ_THREADS) Ga[e] = 0.0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (q + 8 * u < NT) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = ti[u] * 16 + lk + 4 * v, c = tj[u] * 16 + li;
                    if (r < w && c < w) {
                        Ga[c * PQ_GP + r] = acc[u][v];
                        Ga[r * PQ_GP + c] = acc[u][v];
                    }
                }
            }
        }
        __syncthreads();
        // diagonal, trace and (first pass) the shift
        double trl = 0.0;
        if (tid < 128) {
            const double g = tid < w ? Ga[tid * PQ_GP + tid] : 0.0;
            d0[tid] = g;
            trl = g;
        }
        trl = wave_sum(trl);
        if (lane == 0) s_tr[q] = trl;
        if (tid == 0) s_fail = 0;
        __syncthreads();
        if (pass == 1) {
            const double tr = s_tr[0] + s_tr[1];
            const double shift = 11.0 * ((double)h * w + (double)w * (w + 1)) * kEps * tr;
            if (tid < w && d0[tid] > 0.0) Ga[tid * PQ_GP + tid] += shift;
            __syncthreads();
        }
        // ---- Cholesky by elimination: lane = row (two halves), wave = 16 columns
        double x[2][16];
        double dlr[2] = {0.0, 0.0}, d0l[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int r = lane + 64 * hh;
            d0l[hh] = r < w ? d0[r] : 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int c = 16 * q + k;
                x[hh][k] = (r < w && c < w) ? Ga[c * PQ_GP + r] : 0.0;
            }
        }
        __syncthreads();                          // G read before the multipliers overwrite it
        bool failed = false;
        double rho = 1.0;
        const double thresh = pass == 1 ? 0.0 : 1e-14;
        double* Lm = Ga;
        pq_steps<0>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if (w > 16) pq_steps<16>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if (w > 32) pq_steps<32>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if (w > 48) pq_steps<48>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if (w > 64) pq_steps<64>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if (w > 80) pq_steps<80>(x, dlr, failed, rho, w, q, lane, d0l, thresh, Lm);
        if ((lane >> 4) == (q & 3)) {             // the owner lanes of this wave's 16 steps
            const int r = 16 * q + (lane & 15);
            if (r < w && r < 128) dl[r] = q < 4 ? dlr[0] : dlr[1];
        }
        if (failed) s_fail = 1;
        if (lane == 0) s_rho[q] = rho;            // rho and failed are uniform per wave
        __syncthreads();
        double rmin = 1.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) rmin = fmin(rmin, s_rho[i]);
        const bool done = need_r == kPqrSpanOnly || (pass >= 2 && rmin >= 0.25);
        if (s_fail || (!done && pass == kPanelQrMaxPass)) {
            failed_all = true;
            break;
        }
        // ---- R accumulation: T_p = R_p T_(p-1), R_p(i, k) = sqrt(D_i) m_(k i) right of
        // the diagonal (m_(k i) = Lm[i][k]), sqrt(D_i) on it
        if (need_r == 1) {
            double* Tout = done ? ws + t.r_out : Tbuf + (int64_t)(pass & 1) * w * w;
            const double* Tin = Tbuf + (int64_t)((pass - 1) & 1) * w * w;
            for (int tt = q; tt < NT; tt += 8) {
                int a = 0, rem = tt;
                while (rem >= T - a) { rem -= T - a; ++a; }
                const int r0 = 16 * a, c0 = 16 * (a + rem);
                const int i = r0 + li;
                const double si = i < w ? sqrt(dl[i]) : 0.0;
                v4d c4 = {0.0, 0.0, 0.0, 0.0};
                if (pass == 1) {
                    // T_1 = R_1: rows r0.., columns c0..
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rr = r0 + lk + 4 * v, cc = c0 + li;
                        double val = 0.0;
                        if (rr < w && cc < w) {
                            const double sr = sqrt(dl[rr]);
                            val = cc > rr ? sr * Lm[rr * PQ_GP + cc] : (cc == rr ? sr : 0.0);
                        }
                        c4[v] = val;
                    }
                } else {
                    const int kend = min(c0 + 16, K4);
                    for (int k0 = r0; k0 < kend; k0 += 4) {
                        const int k = k0 + lk;
                        double av = 0.0;
                        if (i < w && k < w) av = k > i ? si * Lm[i * PQ_GP + k] : (k == i ? si : 0.0);
                        const int jc = c0 + li;
                        const double bv = (k < w && jc < w) ? Tin[(int64_t)jc * w + k] : 0.0;
                        c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c4, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = r0 + lk + 4 * v, cc = c0 + li;
                    if (rr < w && cc < w) Tout[(int64_t)cc * w + rr] = c4[v];
                }
            }
            // the lower triangle of the final R is zero
            if (done)
                for (int e = tid; e < w * w; e += PQ_THREADS) {
                    const int cc = e / w, rr = e - cc * w;
                    if (rr > cc) ws[t.r_out + e] = 0.0;
                }
        }
        __syncthreads();                          // the multipliers are read before M overwrites them
        // ---- M = L^-T D^-1/2 into LDS: M(16 q + k, c) = L^-1(c, 16 q + k) / sqrt(D_c)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int c = lane + 64 * hh;
            if (c < w && q < 6) {
                const double dc = dl[c];
                const double rs = dc > 0.0 ? 1.0 / sqrt(dc) : 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int r = 16 * q + k;
                    Ga[c * PQ_GP + r] = r <= c ? x[hh][k] * rs : 0.0;
                }
            }
        }
        __syncthreads();
        // ---- Q = X M, slab by slab (in place when X is Q: a slab is read before it is
        // overwritten, and the slab read ahead is never the one being written)
        const int ntile = 4 * T;                  // 4 row tiles of 16 x T column tiles
        pq_load(X, ldx, h, w, T, 0, pf);
        for (int row0 = 0; row0 < h; row0 += PQ_RS) {
            pq_put(pf, T, Sb);
            __syncthreads();
            if (row0 + PQ_RS < h) pq_load(X, ldx, h, w, T, row0 + PQ_RS, pf);
            for (int tt = q; tt < ntile; tt += 8) {
                const int rt = tt & 3, ct = tt >> 2;
                const int kend = min(16 * (ct + 1), K4);
                v4d c4 = {0.0, 0.0, 0.0, 0.0};
                const double* sa = Sb + lk * PQ_SP + rt * 16 + li;
                const double* mb = Ga + (ct * 16 + li) * PQ_GP + lk;
                for (int k0 = 0; k0 < kend; k0 += 4)
                    c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[k0 * PQ_SP], mb[k0], c4, 0, 0, 0);
                const int cc = ct * 16 + li;
                if (cc < w) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rr = row0 + rt * 16 + lk + 4 * v;
                        if (rr < h) Qd[(int64_t)cc * qld + rr] = c4[v];
                    }
                }
            }
            __syncthreads();
        }
        if (done) break;
    }
    if (tid == 0) iws[t.cq_flag] = failed_all ? 1 : 0;
}

hipError_t prepare_panel_qr_launches() {
    static unsigned long long done = 0;
    return set_lds_limit_once((const void*)k_panel_qr, (int)PQ_LDS_BYTES, &done);
}

hipError_t launch_panel_qr(double* ws, int* iws, const TsqrTask* tasks, int ntasks, int w, int need_r,
                           hipStream_t s, const int* guard, const int* order) {
    if (ntasks <= 0) return hipSuccess;
    if (w < 1 || w > kPanelQrMaxW) return hipErrorInvalidValue;
    if (need_r != 0 && need_r != 1 && need_r != kPqrSpanOnly) return hipErrorInvalidValue;
    hipError_t e = prepare_panel_qr_launches();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_panel_qr, dim3(ntasks), dim3(PQ_THREADS), PQ_LDS_BYTES, s, ws, iws, tasks, w, need_r,
                       guard, order);
    return hipGetLastError();
}

}  // namespace hsvd
