// Tall-skinny Householder QR (TSQR) for h x w panels, w <= 80, chunks of 256 rows
// (w <= 64) or 160 rows (w <= 80).
//
// Factor: each row chunk of `ch` rows is held in registers and reduced by w
// Householder reflectors (LAPACK dlarfg convention: H = I - tau v v^T, v_j = 1,
// R_jj = beta).  The chunk's reflectors go back into the panel; its R, tau and the
// compact-WY factor T (w x w upper triangular, Q = H_0 ... H_{w-1} = I - V T V^T,
// dlarft forward/columnwise) go into the tree storage.  R factors are then merged
// up a tree of fan-in F = 4 (w <= 64; 2 above) by the QR of the stacked children
// [R_0; ...; R_{F-1}] (F w x w); the work-group that finishes last among a node's
// children performs the merge (an atomic counter per node, reset by that group), so
// the whole tree runs in one launch and no group waits on another.  A node with a
// single child takes that child's R unchanged.
//
// Apply: out = Q [X; 0] for the explicit thin factor Q (h x w).  Each chunk's
// group walks from the root to its chunk; at every merged node [X; 0] - V (T (V_top^T X))
// gives the node's F w rows, of which the w rows of the child on the path are kept
// (single-child nodes are skipped); at the chunk the same three small products give
// the output rows.  Optionally adds U1 * Tm (the merge's U1 U_E,top term).
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "house_qr.hpp"
#include "mfma_f64.hpp"

namespace hsvd {

constexpr int TSQR_THREADS = 1024;

// Node slot layout: R (w*w) | V (F w * w, ld F w) | tau (w) | T (w*w), F = tsqr_fanin(w)
__device__ __forceinline__ int64_t slot_tau(int w) { return (int64_t)(tsqr_fanin(w) + 1) * w * w; }
__device__ __forceinline__ int64_t slot_T(int w) { return (int64_t)(tsqr_fanin(w) + 1) * w * w + w; }

// Slot index of tree node (level, idx) given the chunk count and the fan-in.
__device__ __forceinline__ int node_slot(int nch, int F, int level, int idx) {
    int off = 0, n = nch;
    for (int l = 0; l < level; ++l) { off += n; n = (n + F - 1) / F; }
    return off + idx;
}

// Element (i, l) of the reflector block V whose strictly-lower part is stored in
// the column-major array A (ld) with the unit diagonal implicit.
__device__ __forceinline__ double vref(const double* A, int64_t ld, int i, int l) {
    return i == l ? 1.0 : (i > l ? A[(int64_t)l * ld + i] : 0.0);
}

// Factor work-groups: CPL = 2 columns per 16-lane group (each lane reads a pivot
// value once for both of its columns and keeps it in registers): 512 threads x 16
// rows per lane for panels up to 64 columns (256-row chunks), 768 threads x 10 rows
// for panels up to 80 (160-row chunks, 96 columns of capacity).
// The 768-thread variant (3 waves per SIMD, <= 170 registers a lane) keeps no pivot
// values in registers (read twice from LDS instead), which keeps it free of spills.
constexpr int TSQR_CPL = 2;
template <int LANES, int RMAX, int NTHR>
using TsqrQR = HouseQR<LANES, RMAX, true, (NTHR > 512 ? 1 : RMAX), TSQR_CPL, NTHR>;

template <int LANES, int RMAX, int NTHR>
__global__ __launch_bounds__(NTHR) void k_tsqr_factor(double* __restrict__ ws,
                                                              int* __restrict__ iws,
                                                              const TsqrTask* __restrict__ tasks,
                                                              const ChunkRef* __restrict__ chunks,
                                                              int w, int ch, const int* __restrict__ guard) {
    if (guard && *guard) return;                     // a skipped stage (every group returns)
    extern __shared__ double sm[];
    double* T = sm;                                  // w x (w + 1)
    double* tau = T + (int64_t)w * (w + 1);
    double* z = tau + w;                             // 2w
    double* vbuf = z + 2 * w;                        // 2 * LANES * RMAX
    __shared__ int s_go;
    TsqrQR<LANES, RMAX, NTHR> q;
    constexpr int NG = TsqrQR<LANES, RMAX, NTHR>::NG;

    const ChunkRef cr = chunks[blockIdx.x];
    const TsqrTask t = tasks[cr.task];
    if (t.cq_flag >= 0 && iws[t.cq_flag] == 0) return;          // the Cholesky QR stood
    const int tid = threadIdx.x, nth = blockDim.x;
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    double* P = ws + t.p_off;
    double* store = ws + t.store_off;
    const int64_t S = tsqr_slot_size(w);

    const int F = tsqr_fanin(w);
    int level = 0, idx = cr.chunk, n = t.nch;
    int cur_rows = rows;                // rows of the block in registers
    double* dst = store + S * node_slot(t.nch, F, 0, cr.chunk);
    q.load(P + row0, t.p_ld, rows, w);
    // One factorization call site (the chunk, then each merge this group performs):
    // a single inlined copy keeps the register block free of spills.
    for (;;) {
        q.factor(cur_rows, w, T, tau, z, vbuf);
        if (level == 0) q.store(P + row0, t.p_ld, rows, w);      // chunk reflectors
        else q.store(dst + w * w, F * w, F * w, w);               // rows past the stack are zeros
        q.store_r(dst, cur_rows, w);
        for (int e = tid; e < w * w; e += nth) {
            const int j = e / w, i = e - j * w;
            dst[slot_T(w) + e] = T[(int64_t)j * (w + 1) + i];
        }
        for (int j = tid; j < w; j += nth) dst[slot_tau(w) + j] = tau[j];
        // climb: single-child parents take the R unchanged; at a merged parent the
        // last child to arrive stacks the children's R factors and factors them
        int nsib = 1, parent = 0;
        while (n > 1) {
            parent = idx / F;
            nsib = min(F, n - parent * F);
            dst = store + S * node_slot(t.nch, F, level + 1, parent);
            ++level;
            idx = parent;
            n = (n + F - 1) / F;
            if (nsib > 1) break;
            __syncthreads();
            q.store_r(dst, cur_rows, w);
        }
        if (nsib == 1) break;                                       // reached the root
        if (!tree_arrive(&iws[t.cnt_off + node_slot(t.nch, F, level, parent)], nsib, &s_go))
            return;                                                 // a later sibling merges
        {
            // the children are consecutive slots of the level below
            const double* c0 = store + S * node_slot(t.nch, F, level - 1, parent * F);
            const int gl = tid % LANES;
            const int rlim = nsib * w;
#pragma unroll
            for (int sl = 0; sl < TSQR_CPL; ++sl) {
                const int c = tid / LANES + sl * NG;
#pragma unroll
                for (int tt = 0; tt < RMAX; ++tt) {
                    const int r = gl + LANES * tt;
                    const int ch_i = r / w;
                    q.x[sl * RMAX + tt] =
                        (c < w && r < rlim) ? c0[S * ch_i + (int64_t)c * w + (r - ch_i * w)] : 0.0;
                }
            }
        }
        cur_rows = nsib * w;
    }
    q.store_r(ws + t.r_out, cur_rows, w);
}

// Dense copy of rows [r0, r0 + nrows) of the reflector block V (unit diagonal,
// zeros above) into LDS as Vs[l * ldvs + (i - r0)].
__device__ void stage_v(const double* V, int64_t ldv, int r0, int nrows, int w, double* Vs,
                        int ldvs) {
    for (int e = threadIdx.x; e < nrows * w; e += blockDim.x) {
        const int l = e / nrows, i = e - l * nrows;
        Vs[(int64_t)l * ldvs + i] = vref(V, ldv, r0 + i, l);
    }
}

// One compact-WY level on LDS operands: W = T (V_top^T X), on the matrix cores.  V_top
// is staged in Vs with leading dimension w + 1; X and W have leading dimension w + 1
// (odd pitches keep a fragment's 16 lanes on distinct banks); T is col-major with
// leading dimension w, in LDS (Ts, copied here while the first product runs) or, when
// it does not fit, read from global memory (Tg).  W = T W runs through registers: a
// wave keeps its (at most kApplyKeep) 16 x 16 tiles across the barrier.
constexpr int kApplyKeep = 2;
__device__ void wy_w(const double* Vs, const double* Tg, double* Ts, const double* X, double* W,
                     int w, int c) {
    if (Ts)
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) Ts[e] = Tg[e];
    const int ld = w + 1;
    mfma_small(w, c, w, [&](int l, int i) { return Vs[(int64_t)l * ld + i]; },
               [&](int i, int cc) { return X[(int64_t)cc * ld + i]; },
               [&](int l, int cc, double v) { W[(int64_t)cc * ld + l] = v; });
    __syncthreads();
    const double* T = Ts ? Ts : Tg;
    v4d keep[kApplyKeep];
    mfma_small_keep(w, c, w, [&](int i, int l) { return T[(int64_t)l * w + i]; },
                    [&](int l, int cc) { return W[(int64_t)cc * ld + l]; }, keep);
    __syncthreads();
    mfma_small_store(w, c, keep, [&](int i, int cc, double v) { W[(int64_t)cc * ld + i] = v; });
    __syncthreads();
}

// LDS of the apply (doubles): X ((w + 1) c) | W ((w + 1) c) | Vs (max(w (w + 1),
// kApplySlab ch)) | Ts (w w, only when the whole fits).
constexpr int kApplySlab = 16;          // reflector / U1 columns per staged slab
constexpr int kApplyTiles = 5;          // 16 x 16 chunk-output tiles per wave (ch c <= 5 * 16 * 256)
constexpr size_t kApplyLdsMax = 160 * 1024;
__host__ __device__ inline size_t apply_buf(int w, int ch) {
    const size_t a = (size_t)w * (w + 1), b = (size_t)kApplySlab * ch;
    return a > b ? a : b;
}
__host__ __device__ inline bool apply_stage_t(int w, int ch, int c) {
    return sizeof(double) * (2 * (size_t)(w + 1) * c + apply_buf(w, ch) + (size_t)w * w + 32) <= kApplyLdsMax;
}

__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr_apply(double* __restrict__ ws,
                                                             const int* __restrict__ iws,
                                                             const TsqrTask* __restrict__ tsqr,
                                                             const ApplyTask* __restrict__ tasks,
                                                             const ChunkRef* __restrict__ chunks,
                                                             int w, int ch, int c,
                                                             const int* __restrict__ guard) {
    if (guard && *guard) return;                     // a skipped stage (every group returns)
    extern __shared__ double sm[];
    const int ld = w + 1;
    double* X = sm;                                  // w x c (ld w + 1)
    double* W = X + (int64_t)ld * c;                 // w x c (ld w + 1)
    double* Vs = W + (int64_t)ld * c;                // staged reflector rows (ld w + 1) / slabs
    double* Ts = apply_stage_t(w, ch, c) ? Vs + apply_buf(w, ch) : nullptr;   // T (w x w)
    const ChunkRef cr = chunks[blockIdx.x];
    const ApplyTask a = tasks[cr.task];
    const TsqrTask t = tsqr[a.tsqr];
    if (t.cq_flag >= 0 && iws[t.cq_flag] == 0) return;          // the Cholesky QR stood
    const int tid = threadIdx.x, nth = blockDim.x;
    const double* store = ws + t.store_off;
    const int64_t S = tsqr_slot_size(w);

    const double* Xg = ws + a.x_off;
    for (int e = tid; e < w * c; e += nth) {
        const int cc = e / w, i = e - cc * w;
        X[(int64_t)cc * ld + i] = Xg[e];
    }
    const int F = tsqr_fanin(w);
    const int levels = tsqr_levels(t.nch, F);
    for (int level = levels; level >= 1; --level) {
        int span = 1, nbelow = t.nch;                 // chunks per node one level down; nodes there
        for (int l = 1; l < level; ++l) { span *= F; nbelow = (nbelow + F - 1) / F; }
        const int idx = cr.chunk / (span * F);
        const int pos = (cr.chunk / span) % F;        // which child leads towards this chunk
        if (min(F, nbelow - idx * F) == 1) continue;  // a lone child: the parent is its R
        const bool right = pos > 0;
        const double* slot = store + S * node_slot(t.nch, F, level, idx);
        const double* V = slot + w * w;              // F w x w, ld F w
        __syncthreads();
        stage_v(V, F * w, 0, w, w, Vs, ld);
        __syncthreads();
        wy_w(Vs, slot + slot_T(w), Ts, X, W, w, c);
        if (right) {
            stage_v(V, F * w, pos * w, w, w, Vs, ld);
            __syncthreads();
        }
        // X <- (first child: X, others: 0) - V_child W; each element is read and written
        // by the lane that computes it
        mfma_small(w, c, w, [&](int i, int l) { return Vs[(int64_t)l * ld + i]; },
                   [&](int l, int cc) { return W[(int64_t)cc * ld + l]; },
                   [&](int i, int cc, double v) {
                       double* xp = X + (int64_t)cc * ld + i;
                       *xp = (right ? 0.0 : *xp) - v;
                   });
    }
    // chunk level: out = [X; 0] - V (T (V_top^T X)) over the chunk rows (+ U1 Tm)
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    const double* Vc = ws + t.p_off + row0;
    const int64_t ldv = t.p_ld;
    const double* cslot = store + S * node_slot(t.nch, F, 0, cr.chunk);
    const int vtop = rows < w ? rows : w;
    __syncthreads();
    stage_v(Vc, ldv, 0, vtop, w, Vs, ld);
    for (int e = tid; e < (w - vtop) * w; e += nth) {     // rows past a short chunk: zero
        const int l = e / (w - vtop), i = vtop + e - l * (w - vtop);
        Vs[(int64_t)l * ld + i] = 0.0;
    }
    __syncthreads();
    wy_w(Vs, cslot + slot_T(w), Ts, X, W, w, c);
    double* out = ws + a.out_off;
    const double* U1 = a.add_u_off >= 0 ? ws + a.add_u_off : nullptr;
    const int aw = U1 ? a.add_w : 0;
    const double* Tm = U1 ? ws + a.add_t_off : nullptr;    // aw x c, ld aw
    if (U1 && Ts && aw * c <= w * w) {                      // T is done with: Tm takes its place
        for (int e = tid; e < aw * c; e += nth) Ts[e] = Tm[e];
        Tm = Ts;
    }
    // One product over K = w + aw: out = [X; 0] - [V_chunk | U1] [W; -Tm].  The left
    // operand streams through LDS in slabs of kApplySlab columns, each loaded by all
    // threads at once (coalesced, one memory round trip per slab); the right operand
    // is in LDS (W; Tm when it fit).  Each wave accumulates its 16 x 16 output tiles
    // (tile q = wave + nw u) on the matrix cores across the slabs.
    const int K = w + aw;
    double* Bs = Vs;                                        // slab: Bs[kk * rows + i]
    const int lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (rows + 15) / 16, tn = (c + 15) / 16, ntile = tm * tn;
    v4d acc[kApplyTiles];
#pragma unroll
    for (int u = 0; u < kApplyTiles; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += kApplySlab) {
        const int ks = min(kApplySlab, K - k0);
        __syncthreads();                                    // the previous slab is consumed
        for (int e = tid; e < ks * rows; e += nth) {
            const int kk = e / rows, i = e - kk * rows, k = k0 + kk;
            double v;
            if (k < w) v = (i == k) ? 1.0 : (i > k ? Vc[(int64_t)k * ldv + i] : 0.0);
            else v = U1[(int64_t)(k - w) * a.add_u_ld + row0 + i];
            Bs[(int64_t)kk * rows + i] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kApplyTiles; ++u) {
            const int q = wave + nw * u;
            if (q >= ntile) break;
            const int i0 = (q % tm) * 16, j0 = (q / tm) * 16;
            const int ia = min(i0 + li, rows - 1), jb = min(j0 + li, c - 1);
            const bool iok = i0 + li < rows, jok = j0 + li < c;
#pragma unroll
            for (int q4 = 0; q4 < kApplySlab / 4; ++q4) {
                const int kk = 4 * q4 + lk, k = k0 + kk;
                const bool kok = kk < ks;
                const int kkc = kok ? kk : 0;
                const double av = Bs[(int64_t)kkc * rows + ia];
                const int kb = kok ? k : 0;
                const double bv = kb < w ? W[(int64_t)jb * ld + kb] : -Tm[(int64_t)jb * aw + (kb - w)];
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((iok && kok) ? av : 0.0,
                                                              (jok && kok) ? bv : 0.0, acc[u], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kApplyTiles; ++u) {
        const int q = wave + nw * u;
        if (q >= ntile) break;
        const int i0 = (q % tm) * 16, j0 = (q / tm) * 16, j = j0 + li;
        if (j >= c) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + lk + 4 * v;
            if (i < rows) {
                const double x = (i < w) ? X[(int64_t)j * ld + i] : 0.0;
                out[(int64_t)j * a.out_ld + row0 + i] = x - acc[u][v];
            }
        }
    }
}

template <int LANES, int RMAX, int NTHR>
static hipError_t launch_factor_t(double* ws, int* iws, const TsqrTask* tasks,
                                  const ChunkRef* chunks, int nchunks, int w, int ch, hipStream_t s,
                                  const int* guard) {
    if (w > TsqrQR<LANES, RMAX, NTHR>::WMAX) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * (TsqrQR<LANES, RMAX, NTHR>::lds_doubles(w) + 32);
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_factor<LANES, RMAX, NTHR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tsqr_factor<LANES, RMAX, NTHR>), dim3(nchunks), dim3(NTHR), lds, s, ws,
                       iws, tasks, chunks, w, ch, guard);
    return hipGetLastError();
}

hipError_t launch_tsqr_factor(double* ws, int* iws, const TsqrTask* tasks, const ChunkRef* chunks,
                              int nchunks, int w, int ch, hipStream_t s, const int* guard) {
    if (nchunks <= 0) return hipSuccess;
    if (w < 1 || w > kTsqrMaxW || ch != tsqr_chunk_rows(w)) return hipErrorInvalidValue;
    // a chunk and a stacked pair of R factors must fit the register block
    if (w <= 64) {
        if (ch > 16 * 16 || tsqr_fanin(w) * w > 16 * 16) return hipErrorInvalidValue;
        return launch_factor_t<16, 16, 512>(ws, iws, tasks, chunks, nchunks, w, ch, s, guard);
    }
    if (ch > 16 * 10 || tsqr_fanin(w) * w > 16 * 10) return hipErrorInvalidValue;
    return launch_factor_t<16, 10, 768>(ws, iws, tasks, chunks, nchunks, w, ch, s, guard);
}

hipError_t launch_tsqr_apply(double* ws, const int* iws, const TsqrTask* tsqr, const ApplyTask* tasks,
                             const ChunkRef* chunks, int nchunks, int w, int ch, int c,
                             hipStream_t s, const int* guard) {
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (2 * (size_t)(w + 1) * c + apply_buf(w, ch) +
                                         (apply_stage_t(w, ch, c) ? (size_t)w * w : 0) + 32);
    if (lds > kApplyLdsMax) return hipErrorInvalidValue;
    // wy_w keeps at most kApplyKeep 16 x 16 tiles per wave across its barrier; the chunk
    // product accumulates at most kApplyTiles per wave
    const int nwave = TSQR_THREADS / 64;
    if (((w + 15) / 16) * ((c + 15) / 16) > kApplyKeep * nwave ||
        ((ch + 15) / 16) * ((c + 15) / 16) > kApplyTiles * nwave)
        return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tsqr_apply, dim3(nchunks), dim3(TSQR_THREADS), lds, s, ws, iws, tsqr, tasks,
                       chunks, w, ch, c, guard);
    return hipGetLastError();
}

}  // namespace hsvd
