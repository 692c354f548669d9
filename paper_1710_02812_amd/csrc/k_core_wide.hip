// One-sided (Hestenes) Jacobi SVD of cores wider than the LDS holds: 129 to 160
// columns, i.e. the merge matrix E = [[S1, C S2], [0, R S2]] of two children of rank up
// to 80 (Section 3, the 2k x 2k core of a merge), or a dense or triangular core of that
// size.
//
// A 160 x 160 float64 core is 205 KB, beyond the 160 KB of LDS.  Its columns live in a
// scratch panel of the task in global memory (kWideCoreRows rows per column, zero
// padded; the panel stays in L2 while its work-group runs).  Every sweep visits each
// column pair once, in three phases over X = columns [0, mx) and Y = [mx, nc),
// mx = ceil(nc / 2):
//   1. X against Y: Y in LDS, X columns 0..63 in registers (16-lane group g holds
//      column g) and the rest in a second LDS area (group g also works column g + 64);
//      in round r column j of X meets column (j + r) mod mx of Y (no partner when that
//      index is past Y's end), so the pairs of a round are disjoint;
//   2. Y among itself, in LDS, by recursive halving: a team [lo, hi) splits into
//      A = [lo, lo + m) and B = [lo + m, hi), m = ceil((hi - lo) / 2); for m rounds
//      group j of the team keeps a = lo + j in registers and meets b = lo + m +
//      (j + r) mod m; A and B are the teams of the next depth;
//   3. X among itself, likewise, once X is copied into LDS.
// A pair is rotated when (g_a . g_b)^2 > tol^2 |g_a|^2 |g_b|^2, the threshold of the
// LDS-resident cores; the sweeps stop after one that rotates nothing (or at the sweep
// cap).  The column norms are the singular values; they are sorted, the rank rule
// picks r, and the normalised left vectors are written as by the LDS-resident cores.
// As there, a core that wants only left vectors is first replaced by L of G = L Q (a
// Householder QR of G^T held in registers, three of its columns per 16-lane group):
// L has G's left singular pairs and columns far closer to orthogonal, which about
// halves the sweeps of a merge core.  No skipped set and no right vectors here.
#include "core_common.hpp"
#include "house_qr.hpp"

namespace hsvd {

namespace {

constexpr int WR = kWideCoreRows;       // rows per column (zero padded)
constexpr int WC = kWideCoreMaxN;       // columns at most
constexpr int WTEAM = (WC + 1) / 2;     // columns of the LDS team buffer
constexpr int WLD = WR + 1;             // LDS pitch (doubles)
constexpr int WT = WR / 16;             // rows per lane of a 16-lane group
constexpr int WXE = WTEAM - 64;         // X columns of phase 1 beyond the 64 groups
static_assert(WR % 16 == 0 && WTEAM > 64 && WTEAM <= 2 * 64, "wide core layout");

size_t wide_lds() {
    return sizeof(double) * ((size_t)(WTEAM + WXE) * WLD + 2 * (size_t)WC) + sizeof(int) * (size_t)WC;
}

// Rotates column a (registers ra, squared norm da) against column b (LDS at gb, squared
// norm *dbp) when their cosine exceeds the threshold.  All 16 lanes of a group call it
// with the same `valid`; returns whether it rotated.
__device__ __forceinline__ bool wide_pair(double (&ra)[WT], double& da, double* gb, double* dbp, bool valid,
                                          double tol2) {
    const int gl = threadIdx.x & 15;
    double rb[WT];
    double c0 = 0.0, c1 = 0.0, db = 0.0;
    if (valid) {
        db = *dbp;
#pragma unroll
        for (int t = 0; t < WT; ++t) rb[t] = gb[gl + 16 * t];
#pragma unroll
        for (int t = 0; t < WT; ++t) {
            if (t & 1) c1 = fma(ra[t], rb[t], c1);
            else c0 = fma(ra[t], rb[t], c0);
        }
    }
    const double c = group_sum(c0 + c1, 16);
    if (valid && da > 0.0 && db > 0.0 && c * c > tol2 * da * db) {
        double cs, sn, tt;
        jacobi_rotation(da, db, c, cs, sn, tt);
#pragma unroll
        for (int t = 0; t < WT; ++t) {
            const double xa = ra[t];
            ra[t] = cs * xa - sn * rb[t];
            gb[gl + 16 * t] = sn * xa + cs * rb[t];
        }
        if (gl == 0) *dbp = db + tt * c;
        da = da - tt * c;
        return true;
    }
    return false;
}

// One recursive-halving tournament over the tn <= WTEAM columns of the LDS team buffer
// (column s at Ls + s WLD, squared norm dn[s]); called by the whole work-group (64
// groups cover every depth for tn <= 80).  Returns whether this thread's group rotated.
__device__ bool wide_team(double* Ls, double* dn, int tn, double tol2) {
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
    bool rot = false;
    for (int dep = 0; ((tn + (1 << dep) - 1) >> dep) >= 2; ++dep) {
        const int gpt = (tn + (2 << dep) - 1) >> (dep + 1);     // groups (and rounds) per team
        const int tm = grp / gpt, j = grp - tm * gpt;
        int lo = 0, hi = tn;
        for (int i = 0; i < dep; ++i) {
            const int m = (hi - lo + 1) >> 1;
            if ((tm >> (dep - 1 - i)) & 1) lo += m;
            else hi = lo + m;
        }
        const int m = (hi - lo + 1) >> 1;
        const bool act = tm < (1 << dep) && hi - lo >= 2 && j < m;
        const int a = act ? lo + j : 0;
        double ra[WT];
        double da = 0.0;
        if (act) {
            da = dn[a];
#pragma unroll
            for (int t = 0; t < WT; ++t) ra[t] = Ls[a * WLD + gl + 16 * t];
        }
        bool moved = false;
        int bi = j;                                               // (j + r) mod m
        for (int r = 0; r < gpt; ++r, bi = (bi + 1 == m) ? 0 : bi + 1) {
            const int b = act ? lo + m + bi : 0;
            const bool valid = act && r < m && b < hi;
            if (wide_pair(ra, da, Ls + (valid ? b : 0) * WLD, dn + (valid ? b : 0), valid, tol2)) moved = true;
            __syncthreads();
        }
        if (moved) {
#pragma unroll
            for (int t = 0; t < WT; ++t) Ls[a * WLD + gl + 16 * t] = ra[t];
            if (gl == 0) dn[a] = da;
        }
        rot = rot || moved;
        __syncthreads();
    }
    return rot;
}

__global__ __launch_bounds__(CORE_THREADS) void k_core_wide(double* __restrict__ ws, int* __restrict__ iws,
                                                            const CoreTask* __restrict__ tasks, int maxdim,
                                                            int max_sweeps, unsigned* __restrict__ flags,
                                                            const int* __restrict__ guard) {
    if (guard && *guard) return;                  // a skipped stage (every group returns)
    extern __shared__ double sm[];
    double* L = sm;                               // team buffer: WTEAM columns, pitch WLD
    double* XE = L + (size_t)WTEAM * WLD;         // phase 1: X columns 64.. (WXE of them)
    double* d = XE + (size_t)WXE * WLD;           // squared column norms, then norms
    double* sig = d + WC;
    int* perm = (int*)(sig + WC);
    __shared__ int s_nc, s_r1, s_r2, s_bad, s_rot, s_rank;
    const CoreTask t = tasks[blockIdx.x];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane64 = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const int grp = tid >> 4, gl = tid & 15;
    double* S = ws + t.scr_off;                   // column j at S + j WR

    if (tid == 0) {
        int nc, r1 = 0, r2 = 0;
        if (t.mode == CORE_MERGE) {
            r1 = iws[t.rank1];
            r2 = iws[t.rank2];
            nc = r1 + r2;
        } else {
            nc = (t.rank_in >= 0) ? iws[t.rank_in] : t.dim;
        }
        if (nc > maxdim) nc = maxdim;
        if (nc > WC) nc = WC;
        s_nc = nc; s_r1 = r1; s_r2 = r2; s_bad = 0;
    }
    __syncthreads();
    const int nc = s_nc, nr = nc, r1 = s_r1;

    // ---- the core into the scratch panel, rows past nr zero
    int bad = 0;
    for (int e = tid; e < nc * WR; e += nth) {
        const int j = e / WR, i = e - j * WR;
        double v = 0.0;
        if (i < nr) {
            if (t.mode == CORE_UPPER) {
                v = (i <= j) ? ws[t.m_off + (int64_t)j * t.m_ld + i] : 0.0;
            } else if (t.mode == CORE_UPPER_T) {
                v = (j <= i) ? ws[t.m_off + (int64_t)i * t.m_ld + j] : 0.0;
            } else if (t.mode == CORE_DENSE) {
                v = ws[t.m_off + (int64_t)j * t.m_ld + i];
            } else if (j < r1) {
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
        S[(int64_t)j * WR + i] = v;
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();

    // ---- LQ preconditioning: row c of G (column c of G^T) in slot c / 64 of group c % 64,
    // lane rows are G's columns; G^T = Q R leaves R in the registers and L = R^T goes
    // back to the panel.  Scratch: tau -> sig, the pivot buffers -> the team buffer.
    if (t.precond && !s_bad && nc > 1) {
        using QR = HouseQR<16, WT, false, 16, 3, CORE_THREADS>;
        static_assert(QR::WMAX >= WC && QR::VB == WR, "preconditioner layout");
        QR q;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int c = q.col_of(s);
#pragma unroll
            for (int u = 0; u < WT; ++u) {
                const int r = gl + 16 * u;
                q.x[s * WT + u] = (c < nr && r < nc) ? S[(int64_t)r * WR + c] : 0.0;
            }
        }
        q.factor(nc, nr, d, sig, d, L);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int c = q.col_of(s);
#pragma unroll
            for (int u = 0; u < WT; ++u) {
                const int r = gl + 16 * u;
                if (r < nc && c < WR) S[(int64_t)r * WR + c] = (r <= c) ? q.x[s * WT + u] : 0.0;
            }
        }
        __syncthreads();
    }

    const double tol = t.orth_tol > 0.0 ? t.orth_tol : (double)(nr > 1 ? nr : 1) * kEps;
    const double tol2 = tol * tol;
    const int mx = (nc + 1) >> 1, my = nc - mx;
    bool converged = (nc <= 1) || s_bad;
    int sweep = 0;
    for (; !converged && sweep < max_sweeps; ++sweep) {
        for (int j = wave; j < nc; j += nw) {
            double s = 0.0;
            for (int i = lane64; i < nr; i += 64) {
                const double g = S[(int64_t)j * WR + i];
                s = fma(g, g, s);
            }
            s = wave_sum(s);
            if (lane64 == 0) d[j] = s;
        }
        __syncthreads();
        // (every thread read the previous sweep's flag before the barrier above)
        if (tid == 0) s_rot = 0;
        bool rot = false;

        // phase 1: X (registers and the XE area) against Y (LDS)
        {
            const int j0 = grp, j1 = grp + 64;
            const bool h0 = j0 < mx, h1 = j1 < mx;
            double rx0[WT];
            double dx0 = 0.0, dx1 = 0.0;
            if (h0) {
                dx0 = d[j0];
#pragma unroll
                for (int u = 0; u < WT; ++u) rx0[u] = S[(int64_t)j0 * WR + gl + 16 * u];
            }
            if (h1) dx1 = d[j1];
            for (int e = tid; e < my * WR; e += nth) {
                const int j = e / WR, i = e - j * WR;
                L[j * WLD + i] = S[(int64_t)(mx + j) * WR + i];
            }
            for (int e = tid; e < (mx - 64) * WR; e += nth) {
                const int j = e / WR, i = e - j * WR;
                XE[j * WLD + i] = S[(int64_t)(64 + j) * WR + i];
            }
            __syncthreads();
            double* xa = XE + (h1 ? j1 - 64 : 0) * WLD;
            int b0 = h0 ? j0 : 0, b1 = h1 ? j1 : 0;                 // (j + r) mod mx
            for (int r = 0; r < mx; ++r) {
                const bool v0 = h0 && b0 < my, v1 = h1 && b1 < my;
                if (wide_pair(rx0, dx0, L + (v0 ? b0 : 0) * WLD, d + mx + (v0 ? b0 : 0), v0, tol2)) rot = true;
                double ra1[WT];
#pragma unroll
                for (int u = 0; u < WT; ++u) ra1[u] = v1 ? xa[gl + 16 * u] : 0.0;
                if (wide_pair(ra1, dx1, L + (v1 ? b1 : 0) * WLD, d + mx + (v1 ? b1 : 0), v1, tol2)) {
                    rot = true;
#pragma unroll
                    for (int u = 0; u < WT; ++u) xa[gl + 16 * u] = ra1[u];
                }
                __syncthreads();
                b0 = (b0 + 1 == mx) ? 0 : b0 + 1;
                b1 = (b1 + 1 == mx) ? 0 : b1 + 1;
            }
            if (h0) {
#pragma unroll
                for (int u = 0; u < WT; ++u) S[(int64_t)j0 * WR + gl + 16 * u] = rx0[u];
                if (gl == 0) d[j0] = dx0;
            }
            if (h1 && gl == 0) d[j1] = dx1;
            for (int e = tid; e < (mx - 64) * WR; e += nth) {
                const int j = e / WR, i = e - j * WR;
                S[(int64_t)(64 + j) * WR + i] = XE[j * WLD + i];
            }
        }

        // phase 2: Y among itself (still in LDS), then back to the panel
        if (wide_team(L, d + mx, my, tol2)) rot = true;
        for (int e = tid; e < my * WR; e += nth) {
            const int j = e / WR, i = e - j * WR;
            S[(int64_t)(mx + j) * WR + i] = L[j * WLD + i];
        }
        __syncthreads();

        // phase 3: X among itself
        for (int e = tid; e < mx * WR; e += nth) {
            const int j = e / WR, i = e - j * WR;
            L[j * WLD + i] = S[(int64_t)j * WR + i];
        }
        __syncthreads();
        if (wide_team(L, d, mx, tol2)) rot = true;
        for (int e = tid; e < mx * WR; e += nth) {
            const int j = e / WR, i = e - j * WR;
            S[(int64_t)j * WR + i] = L[j * WLD + i];
        }
        if (rot) s_rot = 1;
        __syncthreads();
        if (s_rot == 0) converged = true;
    }
    if (tid == 0 && flags) {
        unsigned f = 0;
        if (s_bad) f |= 1u;
        if (!converged) f |= 2u;
        if (f) atomicOr(flags, f);
        atomicMax(flags + 1, (unsigned)sweep);
    }

    // ---- singular values (exact column norms), sorted descending
    for (int j = wave; j < nc; j += nw) {
        double s = 0.0;
        for (int i = lane64; i < nr; i += 64) {
            const double g = S[(int64_t)j * WR + i];
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
    if (wave == 0) {
        const int r = s_bad ? 0 : select_rank(sig, nc, t, iws);
        if (lane64 == 0) {
            s_rank = r;
            if (t.rank_out >= 0) iws[t.rank_out] = r;
        }
    }
    __syncthreads();
    const int r = s_rank;

    // ---- outputs
    for (int i = tid; i < t.out_w; i += nth) ws[t.sig_off + i] = (i < r) ? sig[i] : 0.0;
    if (t.sigall_off >= 0 && t.mode != CORE_MERGE)
        for (int i = tid; i < t.dim; i += nth) ws[t.sigall_off + i] = (i < nc && !s_bad) ? sig[i] : 0.0;
    if (t.mode == CORE_MERGE) {
        const int rowsT = t.t_ld, rowsU = t.u_ld, r2 = s_r2;
        for (int e = tid; e < rowsT * t.out_w; e += nth) {
            const int i = e / rowsT, j = e - i * rowsT;
            ws[t.t_off + (int64_t)i * t.t_ld + j] = (i < r && j < r1) ? S[(int64_t)perm[i] * WR + j] / sig[i] : 0.0;
        }
        for (int e = tid; e < rowsU * t.out_w; e += nth) {
            const int i = e / rowsU, j = e - i * rowsU;
            ws[t.u_off + (int64_t)i * t.u_ld + j] =
                (i < r && j < r2) ? S[(int64_t)perm[i] * WR + r1 + j] / sig[i] : 0.0;
        }
    } else if (t.u_off >= 0) {
        const int rowsU = t.dim;
        for (int e = tid; e < rowsU * t.out_w; e += nth) {
            const int i = e / rowsU, j = e - i * rowsU;
            ws[t.u_off + (int64_t)i * t.u_ld + j] = (i < r && j < nr) ? S[(int64_t)perm[i] * WR + j] / sig[i] : 0.0;
        }
    }
}

}  // namespace

hipError_t prepare_core_wide() {
    static unsigned long long done = 0;
    return set_lds_limit_once((const void*)k_core_wide, (int)wide_lds(), &done);
}

hipError_t launch_core_wide(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                            int max_sweeps, unsigned* flags, hipStream_t s, const int* guard) {
    if (ntasks <= 0) return hipSuccess;
    if (maxdim < 1 || maxdim > WC) return hipErrorInvalidValue;
    hipError_t e = prepare_core_wide();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_core_wide, dim3(ntasks), dim3(CORE_THREADS), wide_lds(), s, ws, iws, tasks, maxdim,
                       max_sweeps, flags, guard);
    return hipGetLastError();
}

}  // namespace hsvd
