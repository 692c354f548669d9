// Pieces shared by the one-sided Jacobi cores (the LDS-resident cores of at most 128
// columns and the wide merge cores of at most 160): the rotation of one column pair and
// the truncation rank of the sorted singular values.
#pragma once
#include "hsvd_internal.hpp"
#include "device_common.hpp"

namespace hsvd {

constexpr int CORE_THREADS = 1024;

// First index i < nc where pred(i) fails, else nc; called by a whole wave.
template <typename F>
__device__ __forceinline__ int wave_first_fail(int nc, F pred) {
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < nc; base += 64) {
        const unsigned long long f = __ballot(base + lane < nc && !pred(base + lane));
        if (f) return base + __builtin_ctzll(f);
    }
    return nc;
}

// The truncation rank of sorted values sig (descending), for one wave: a zero floor
// of max(rows, cols) eps sig_0, then the task's rule; at most kcap.
__device__ inline int select_rank(const double* sig, int nc, const CoreTask& t, const int* iws) {
    if (nc == 0) return 0;
    const double s0 = sig[0];
    if (!(s0 > 0.0)) return 0;
    const int fr = t.floor_rows;
    const int fc = t.floor_cols < 0 ? nc : t.floor_cols;
    const double floor = (double)(fr > fc ? fr : fc) * kEps * s0;
    const int nonzero = wave_first_fail(nc, [&](int i) { return sig[i] > floor; });
    int r;
    if (t.fixed_rank_slot >= 0) {
        r = iws[t.fixed_rank_slot];
    } else if (t.rule == 0) {
        const double lim = t.tol * s0;
        r = wave_first_fail(nc, [&](int i) { return sig[i] >= lim; });
    } else {
        // smallest r whose discarded tail sum_{i>=r} s_i^2 is <= tol^2 * total,
        // tails accumulated from the smallest value up (in that order, by one lane)
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
    return r;
}

// The plane rotation that makes columns a and b orthogonal, from their squared norms
// da, db and inner product c: tan of its angle t = sign(dd) g / (|dd| + sqrt(dd^2 + g^2)),
// dd = db - da, g = 2 c (the smaller root of t^2 + 2 (dd / g) t - 1 = 0); then
// a' = cs a - sn b, b' = sn a + cs b, |a'|^2 = da - t c, |b'|^2 = db + t c.
__device__ __forceinline__ void jacobi_rotation(double da, double db, double c, double& cs, double& sn,
                                                double& tt) {
    const double dd = db - da, gg = 2.0 * c;
    if (fmax(fabs(dd), fabs(gg)) < 1e150) {
        // the angle only steers convergence: hardware estimates suffice; orthogonality
        // comes from the refined cs below
        const double x = fma(dd, dd, gg * gg);
        const double hyp = x * __builtin_amdgcn_rsq(x);
        tt = copysign(1.0, dd) * gg * __builtin_amdgcn_rcp(fabs(dd) + hyp);
    } else {
        const double zeta = dd / gg, az = fabs(zeta);
        tt = (az > 1e150) ? 0.5 / zeta : copysign(1.0 / (az + sqrt(1.0 + zeta * zeta)), zeta);
    }
    cs = rsqrt_nr(fma(tt, tt, 1.0));
    sn = cs * tt;
}

}  // namespace hsvd
