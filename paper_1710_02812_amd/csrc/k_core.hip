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
// Each sweep starts with a test on the Gram matrix G^T G (matrix cores): the sweeps
// stop when no pair has |g_a . g_b| > tol * |g_a| |g_b|, and a sweep visits only the
// pairs the test marked (rotating them above half that threshold, so that a marked
// pair near it is not declined on a differently rounded dot product).  When the
// core has more columns than the rank cap, pairs
// whose two columns both had a norm below 1e-3 of the cap-th largest at the start
// of the first sweep are skipped in every sweep: the cap drops such columns
// whatever their mutual rotations, and their rotations against larger columns
// still run.  The set is fixed once: re-deciding it every sweep lets columns of a
// spectrum that decays through the threshold drift in and out of it, which stalls
// convergence.
// Once converged, the skip is accepted only if the kept columns are all large,
// exceed the Frobenius norm of the small ones, and the rank rule provably
// excludes the small part; otherwise full sweeps continue from that state.  At
// convergence G = U S (V not needed for merges, which drop the right factors);
// the optional accumulated rotations give V.
//
// Preconditioning (when only left vectors are wanted): G is first replaced by L
// of G = L Q (a Householder QR of G^T held in registers).  L has the left singular
// pairs of G, and its columns are far closer to orthogonal than those of a merge
// matrix E, whose two halves hold nearly parallel copies of shared directions:
// on merge cores this halves the number of sweeps.
// Columns are then sorted by norm, the truncation rule picks the rank r, and the
// normalised left vectors, singular values and (optionally) V are written.
#include "core_common.hpp"
#include "house_qr.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

// ROWS: every column is padded with zeros to ROWS >= maxdim rows (a multiple of 16)
template <int ROWS>
__global__ __launch_bounds__(CORE_THREADS) void k_core(double* __restrict__ ws, int* __restrict__ iws,
                                                       const CoreTask* __restrict__ tasks,
                                                       int maxdim, int max_sweeps,
                                                       unsigned* __restrict__ flags, int with_v,
                                                       const int* __restrict__ guard) {
    if (guard && *guard) return;                  // a skipped stage (every group returns)
    extern __shared__ double sm[];
    const CoreTask t = tasks[blockIdx.x];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane64 = tid & 63, wave = tid >> 6, nw = nth >> 6;
    static_assert(ROWS % 16 == 0 && ROWS <= 128, "ROWS");
    const int ldg = ROWS + 1;
    double* G = sm;
    double* V = G + (int64_t)maxdim * ldg;
    double* d = V + (with_v ? (int64_t)maxdim * ldg : 0);
    double* sig = d + maxdim + 1;
    int* perm = (int*)(sig + maxdim);
    __shared__ int s_nr, s_nc, s_r1, s_r2, s_rot, s_bad, s_rank, s_safe;
    __shared__ unsigned char sflag[128];
    __shared__ unsigned long long s_mask[2];      // sflag as bits (columns 0..63, 64..127)
    __shared__ unsigned s_pair[128 * 4];          // pair (i < j) still to rotate: bit j % 32 of word 4 i + j / 32
    __shared__ double s_dmax;

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
    // right vectors are accumulated only for cores of at most 96 columns (the launch
    // rejects with_v above that), so the wider variants compile without them
    const bool accv = ROWS <= 96 && (t.v_off >= 0) && with_v;

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
    for (int e = tid; e < nc * (ROWS - nr); e += nth) {
        const int j = e / (ROWS - nr), i = nr + e - j * (ROWS - nr);
        G[(int64_t)j * ldg + i] = 0.0;
    }
    if (accv)
        for (int e = tid; e < nc * ROWS; e += nth) {
            const int j = e / ROWS, i = e - j * ROWS;
            V[(int64_t)j * ldg + i] = (i == j) ? 1.0 : 0.0;
        }
    for (int j = tid; j < 128; j += nth) sflag[j] = 0;
    if (tid < 2) s_mask[tid] = 0ull;
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();

    // ---- LQ preconditioning: G = L Q by Householder QR of G^T; the sweeps then
    // run on L (same left singular pairs).  Row c of G is column c of G^T, held by
    // the 16-lane group c % 64 (two columns per group), lane rows are G's columns;
    // Q is not formed.
    if (t.precond && !accv && !s_bad && nc > 1) {
        constexpr int RQ = ROWS / 16;             // rows of G^T (columns of G) per lane
        using QR = HouseQR<16, RQ, false, 16, 2, CORE_THREADS>;
        static_assert(QR::WMAX >= ROWS && QR::VB == ROWS, "preconditioner layout");
        QR q;
        const int gl = tid & 15;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = q.col_of(s);
#pragma unroll
            for (int u = 0; u < RQ; ++u) {
                const int r = gl + 16 * u;
                q.x[s * RQ + u] = (c < nr && r < nc) ? G[(int64_t)r * ldg + c] : 0.0;
            }
        }
        // scratch: tau -> sig, the two pivot buffers -> the first 2 ROWS entries of G
        // (maxdim >= nc >= 2 here, so G holds >= 2 ROWS + 2); T and z are not used.
        // Columns c >= nr of G^T are zero; only c < ROWS have a row of G.
        __syncthreads();                          // all of G is in registers
        q.factor(nc, nr, G, sig, d, G);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = q.col_of(s);
#pragma unroll
            for (int u = 0; u < RQ; ++u) {
                const int r = gl + 16 * u;
                if (r < nc && c < ROWS) G[(int64_t)r * ldg + c] = (r <= c) ? q.x[s * RQ + u] : 0.0;
            }
        }
        __syncthreads();
    }

    // ---- one-sided Jacobi sweeps
    // Pair order by recursive halving: a team of columns [lo, hi) splits into
    // A = [lo, lo + m) and B = [lo + m, hi), m = ceil((hi - lo) / 2) (B padded with a
    // dummy when odd); for m rounds group j of the team keeps a = lo + j in registers
    // and meets b = lo + m + (j + r) mod m, read from and written back to LDS; then A
    // and B are teams of the next depth, all teams of a depth side by side.  Every pair
    // meets once per sweep in about nc rounds (as the circle method), but only one of
    // its two columns crosses LDS in a round.  Depth d has 2^d teams of at most
    // ceil(nc / 2^d) columns, each given ceil(nc / 2^(d+1)) groups: <= 64 for nc <= 128.
    constexpr int gsz = 16;                         // lanes per pair: 64 groups cover nc <= 128
    const int grp = tid / gsz, gl = tid - grp * gsz;
    constexpr int TMAX = ROWS / gsz;                // rows per lane, unconditional (zero padded)
    const double tol = t.orth_tol > 0.0 ? t.orth_tol : (double)(nr > 1 ? nr : 1) * kEps;
    const double tol2 = tol * tol;
    // skip threshold: squared norm <= (1e-3)^2 of the cap-th largest squared norm
    constexpr double kSkip2 = 1e-6;
    constexpr double kGap2 = 1e-4;
    const int cap_all = (t.fixed_rank_slot >= 0) ? min(t.kcap, iws[t.fixed_rank_slot]) : t.kcap;
    bool converged = (nc <= 1) || s_bad;
    bool skip = true;
    bool classify = true;       // the skipped set is fixed at the first sweep of a phase
    int sweep = 0;
  resume:
    for (; !converged; ++sweep) {
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
        if (classify && wave == 0) {
            // only columns far below the cap-th largest can be left unrotated among
            // themselves: the rank cap drops them whatever their mutual rotations
            double dk = -1.0;
            if (skip && nc > cap_all && cap_all >= 1) {
                for (int j = lane64; j < nc; j += 64) {
                    const double dj = d[j];
                    int pos = 0;
#pragma unroll 8
                    for (int i = 0; i < nc; ++i) {
                        const double di = d[i];
                        pos += (di > dj) || (di == dj && i < j);
                    }
                    if (pos == cap_all - 1) dk = dj;
                }
                dk = wave_max(dk);
            }
            // ... and only when they sit apart from the rest (largest of them at most
            // 1e-2 of the smallest kept norm): a set cut through a cluster of similar
            // norms leaves rotations half done and convergence turns linear
            double mx = 0.0, mn = 1.0e300;
            for (int j = lane64; j < nc; j += 64) {
                const bool sm = (dk >= 0.0) && (d[j] <= kSkip2 * dk);
                if (sm) mx = fmax(mx, d[j]); else mn = fmin(mn, d[j]);
            }
            mx = wave_max(mx);
            mn = -wave_max(-mn);
            const bool apart = mx <= kGap2 * mn;
            const bool on = apart && (dk >= 0.0);
            const bool f0 = on && lane64 < nc && d[lane64] <= kSkip2 * dk;
            const bool f1 = on && lane64 + 64 < nc && d[lane64 + 64] <= kSkip2 * dk;
            sflag[lane64] = f0;
            sflag[lane64 + 64] = f1;
            const unsigned long long b0 = __ballot(f0), b1 = __ballot(f1);
            if (lane64 == 0) { s_mask[0] = b0; s_mask[1] = b1; }
        }
        classify = false;
        for (int e = tid; e < 128 * 4; e += nth) s_pair[e] = 0u;
        __syncthreads();
        const unsigned long long mask0 = s_mask[0], mask1 = s_mask[1];
        // Convergence test on the Gram matrix G^T G of the current columns (float64
        // matrix cores, fragments straight from LDS): a pair still needs a rotation when
        // (g_i . g_j)^2 > tol^2 |g_i|^2 |g_j|^2, the test a round applies.  No such pair
        // (outside the skipped set): converged, without a sweep that rotates nothing.
        // Otherwise the sweep visits only the marked pairs; a pair that a later
        // rotation of the sweep disturbs is caught by the next test.
        {
            const int t16 = (nc + 15) / 16, ntile = t16 * (t16 + 1) / 2;
            const int li = lane64 & 15, lk = lane64 >> 4;
            for (int tt = wave; tt < ntile; tt += nw) {
                int ti = 0, rem = tt;                     // upper triangle of tiles, row by row
                while (rem >= t16 - ti) { rem -= t16 - ti; ++ti; }
                const int tj = ti + rem;
                const int ia = min(ti * 16 + li, nc - 1), jb = min(tj * 16 + li, nc - 1);
                const bool iok = ti * 16 + li < nc, jok = tj * 16 + li < nc;
                const double* gi = G + (int64_t)ia * ldg;
                const double* gj = G + (int64_t)jb * ldg;
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                for (int k0 = 0; k0 < ROWS; k0 += 4) {
                    const double av = gi[k0 + lk], bv = gj[k0 + lk];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(iok ? av : 0.0, jok ? bv : 0.0, acc, 0, 0, 0);
                }
                const int j = tj * 16 + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = ti * 16 + lk + 4 * v;
                    if (i < j && j < nc) {
                        const bool fi = ((i < 64 ? mask0 >> i : mask1 >> (i - 64)) & 1ull) != 0;
                        const bool fj = ((j < 64 ? mask0 >> j : mask1 >> (j - 64)) & 1ull) != 0;
                        const double di = d[i], dj = d[j], c = acc[v];
                        if (!(fi && fj) && di > 0.0 && dj > 0.0 && c * c > tol2 * di * dj) {
                            atomicOr(&s_pair[i * 4 + (j >> 5)], 1u << (j & 31));
                            s_rot = 1;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (s_rot == 0) { converged = true; break; }
        if (sweep >= max_sweeps) break;
        for (int dep = 0; ((nc + (1 << dep) - 1) >> dep) >= 2; ++dep) {
            const int gpt = (nc + (2 << dep) - 1) >> (dep + 1);      // groups (and rounds) per team
            const int tm = grp / gpt, j = grp - tm * gpt;
            int lo = 0, hi = nc;
            for (int i = 0; i < dep; ++i) {
                const int m = (hi - lo + 1) >> 1;
                if ((tm >> (dep - 1 - i)) & 1) lo += m;
                else hi = lo + m;
            }
            const int m = (hi - lo + 1) >> 1;
            const bool act = tm < (1 << dep) && hi - lo >= 2 && j < m;
            const int a = act ? lo + j : 0;
            const bool fa = ((a < 64 ? mask0 >> a : mask1 >> (a - 64)) & 1ull) != 0;
            double* ga = G + (int64_t)a * ldg;
            // a's marks against every column (a < b throughout the depth), in registers;
            // when a is in the skipped set, the other members' marks are cleared
            const unsigned long long sk0 = fa ? mask0 : 0ull, sk1 = fa ? mask1 : 0ull;
            const unsigned pw0 = s_pair[a * 4] & ~(unsigned)sk0, pw1 = s_pair[a * 4 + 1] & ~(unsigned)(sk0 >> 32),
                           pw2 = s_pair[a * 4 + 2] & ~(unsigned)sk1, pw3 = s_pair[a * 4 + 3] & ~(unsigned)(sk1 >> 32);
            double ra[TMAX];
            double da = 0.0;
            if (act) {
                da = d[a];
#pragma unroll
                for (int t = 0; t < TMAX; ++t) ra[t] = ga[gl + t * gsz];
            }
            // the rounds in which this group meets a marked partner, once per depth: bit r
            // for b = lo + m + (j + r) mod m, i.e. the marks of B = [lo + m, hi) (at most
            // m <= 64 columns) rotated by j within m bits
            unsigned long long rmask = 0ull;
            if (act) {
                const unsigned long long lo64 = (unsigned long long)pw0 | ((unsigned long long)pw1 << 32);
                const unsigned long long hi64 = (unsigned long long)pw2 | ((unsigned long long)pw3 << 32);
                const int off = lo + m, nb = hi - off;
                unsigned long long win = off == 0 ? lo64
                                       : off < 64 ? (lo64 >> off) | (hi64 << (64 - off)) : hi64 >> (off - 64);
                if (nb < 64) win &= (1ull << nb) - 1ull;
                rmask = j == 0 ? win : (win >> j) | (win << (m - j));
                if (m < 64) rmask &= (1ull << m) - 1ull;
            }
            bool moved = false;
            int bi = j;                                        // (j + r) mod m
            for (int r = 0; r < gpt; ++r, bi = (bi + 1 == m) ? 0 : bi + 1) {
                const bool valid = ((rmask >> r) & 1ull) != 0;
                const int b = lo + m + bi;
                double rb[TMAX];
                double c0 = 0.0, c1 = 0.0, db = 0.0;
                double* gb = G + (int64_t)(valid ? b : 0) * ldg;
                if (valid) {
                    db = d[b];
#pragma unroll
                    for (int t = 0; t < TMAX; ++t) rb[t] = gb[gl + t * gsz];
#pragma unroll
                    for (int t = 0; t < TMAX; ++t) {          // TMAX may be odd (112 rows)
                        if (t & 1) c1 = fma(ra[t], rb[t], c1);
                        else c0 = fma(ra[t], rb[t], c0);
                    }
                }
                const double c = group_sum(c0 + c1, gsz);
                if (valid) {
                    // a quarter of the test's threshold: the pair was marked on the Gram
                    // value, and c here (a different rounding, running norms) must not
                    // decline the rotation of a pair near the threshold
                    if (da > 0.0 && db > 0.0 && c * c > 0.25 * tol2 * da * db) {
                        double cs, sn, tt;
                        jacobi_rotation(da, db, c, cs, sn, tt);
#pragma unroll
                        for (int t = 0; t < TMAX; ++t) {
                            const double xa = ra[t];
                            ra[t] = cs * xa - sn * rb[t];
                            gb[gl + t * gsz] = sn * xa + cs * rb[t];
                        }
                        if (accv) {
                            double* va = V + (int64_t)a * ldg;
                            double* vb = V + (int64_t)b * ldg;
                            double xa[TMAX], xb[TMAX];
#pragma unroll
                            for (int t = 0; t < TMAX; ++t) {
                                xa[t] = va[gl + t * gsz];
                                xb[t] = vb[gl + t * gsz];
                            }
#pragma unroll
                            for (int t = 0; t < TMAX; ++t) {
                                va[gl + t * gsz] = cs * xa[t] - sn * xb[t];
                                vb[gl + t * gsz] = sn * xa[t] + cs * xb[t];
                            }
                        }
                        if (gl == 0) d[b] = db + tt * c;
                        da = da - tt * c;
                        moved = true;
                    }
                }
                __syncthreads();
            }
            if (moved) {
#pragma unroll
                for (int t = 0; t < TMAX; ++t) ga[gl + t * gsz] = ra[t];
                if (gl == 0) d[a] = da;
            }
            __syncthreads();
        }
    }
    if (tid == 0 && flags) {
        unsigned f = 0;
        if (s_bad) f |= 1u;
        if (!converged) f |= 2u;
        if (f) atomicOr(flags, f);
        atomicMax(flags + 1, (unsigned)sweep);
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
#pragma unroll 8
        for (int i = 0; i < nc; ++i) {
            const double si = d[i];
            pos += (si > sj) || (si == sj && i < j);
        }
        perm[pos] = j;
        sig[pos] = sj;
    }
    __syncthreads();
    if (tid == 0 && t.energy_off >= 0) {
        // captured energy of the sketch against the block's: the leaf keeps too few
        // columns when the part it cannot see exceeds the tolerance
        double cap = 0.0;
        for (int j = 0; j < nc; ++j) cap = fma(sig[j], sig[j], cap);
        const double E = ws[t.energy_off];
        const int miss = (E - cap > t.tol * t.tol * E * (1.0 + 1e-9)) ? 1 : 0;
        iws[t.flag_slot] = miss;
        if (miss && flags) atomicOr(flags, 4u);
    }
    if (wave == 0) {
        const int r = s_bad ? 0 : select_rank(sig, nc, t, iws);
        // accept the skipped small-small rotations only if they cannot change the result
        int safe = 1;
        if (skip && r > 0) {
            // the skipped set (fixed at the first sweep) is S; at convergence every
            // other pair is orthogonal, so the kept columns are exact if none of them
            // is in S and S cannot hold a singular value as large as the r-th
            double small2 = 0.0;
            bool any_small = false, kept_small = false;
            for (int j = lane64; j < nc; j += 64) {
                if (sflag[j]) { small2 = fma(d[j], d[j], small2); any_small = true; }
                if (j < r && sflag[perm[j]]) kept_small = true;
            }
            small2 = wave_sum(small2);
            any_small = __ballot(any_small) != 0ull;
            kept_small = __ballot(kept_small) != 0ull;
            if (any_small) {
                if (kept_small) safe = 0;
                const double sm = sqrt(small2);
                if (!(sm < sig[r - 1])) safe = 0;
                int cap = t.kcap;
                if (t.fixed_rank_slot >= 0) cap = min(cap, iws[t.fixed_rank_slot]);
                if (r < cap) {
                    const int fr = t.floor_rows, fc = t.floor_cols < 0 ? nc : t.floor_cols;
                    const double floor = (double)(fr > fc ? fr : fc) * kEps * sig[0];
                    bool excluded = sm <= floor;
                    if (t.fixed_rank_slot < 0 && t.rule == 0) excluded = excluded || sm < t.tol * sig[0];
                    if (t.fixed_rank_slot < 0 && t.rule == 1) {
                        double all2 = 0.0;
                        for (int j = lane64; j < nc; j += 64) all2 = fma(sig[j], sig[j], all2);
                        excluded = excluded || small2 <= t.tol * t.tol * wave_sum(all2);
                    }
                    if (!excluded) safe = 0;
                }
            }
        }
        if (lane64 == 0) {
            s_rank = r;
            s_safe = safe;
            if (safe && t.rank_out >= 0) iws[t.rank_out] = r;
        }
    }
    __syncthreads();
    if (!s_safe) {                 // redo with full sweeps from the current state
        skip = false;
        classify = true;
        converged = false;
        __syncthreads();
        goto resume;
    }
    const int r = s_rank;

    // ---- outputs
    for (int i = tid; i < t.out_w; i += nth) ws[t.sig_off + i] = (i < r) ? sig[i] : 0.0;
    if (t.sigall_off >= 0 && t.mode != CORE_MERGE)
        for (int i = tid; i < t.dim; i += nth) ws[t.sigall_off + i] = (i < nc && !s_bad) ? sig[i] : 0.0;
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

template <int ROWS>
size_t core_lds(int maxdim, int with_v) {
    return sizeof(double) * ((size_t)maxdim * (ROWS + 1) * (with_v ? 2 : 1) + 2 * (size_t)maxdim + 1) +
           sizeof(int) * maxdim + 64;
}

template <int ROWS>
hipError_t prepare_core_rows() {
    static unsigned long long done = 0;
    return set_lds_limit_once((const void*)k_core<ROWS>, (int)core_lds<ROWS>(ROWS, ROWS <= 96), &done);
}

template <int ROWS>
hipError_t launch_core_rows(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                            int max_sweeps, unsigned* flags, int with_v, hipStream_t s, const int* guard) {
    const size_t lds = core_lds<ROWS>(maxdim, with_v);
    hipError_t e = prepare_core_rows<ROWS>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_core<ROWS>, dim3(ntasks), dim3(CORE_THREADS), lds, s, ws, iws, tasks, maxdim,
                       max_sweeps, flags, with_v, guard);
    return hipGetLastError();
}

hipError_t prepare_core_launches() {
    hipError_t e = prepare_core_rows<32>();
    if (e == hipSuccess) e = prepare_core_rows<64>();
    if (e == hipSuccess) e = prepare_core_rows<96>();
    if (e == hipSuccess) e = prepare_core_rows<112>();
    if (e == hipSuccess) e = prepare_core_rows<128>();
    if (e == hipSuccess) e = prepare_core_wide();
    return e;
}

hipError_t launch_core(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                         int max_sweeps, unsigned* flags, int with_v, hipStream_t s, const int* guard) {
    if (ntasks <= 0) return hipSuccess;
    if (maxdim > kCoreMaxN) {
        if (maxdim > kWideCoreMaxN || with_v) return hipErrorInvalidValue;
        return launch_core_wide(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, s, guard);
    }
    if (maxdim < 1 || (with_v && maxdim > kCoreMaxV)) return hipErrorInvalidValue;
    // rows padded to the smallest variant that holds the largest core of the launch
    if (maxdim <= 32) return launch_core_rows<32>(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, with_v, s, guard);
    if (maxdim <= 64) return launch_core_rows<64>(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, with_v, s, guard);
    if (maxdim <= 96) return launch_core_rows<96>(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, with_v, s, guard);
    if (maxdim <= 112) return launch_core_rows<112>(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, with_v, s, guard);
    return launch_core_rows<128>(ws, iws, tasks, ntasks, maxdim, max_sweeps, flags, with_v, s, guard);
}

}  // namespace hsvd
