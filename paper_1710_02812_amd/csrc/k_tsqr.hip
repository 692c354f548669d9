// Tall-skinny Householder QR (TSQR) for h x w panels, w <= 80, chunks of 256 rows
// (w <= 64) or 160 rows (w <= 80).
//
// Factor: each row chunk of `ch` rows is loaded into LDS and reduced by w
// Householder reflectors (LAPACK dlarfg convention: H = I - tau v v^T, v_j = 1,
// R_jj = beta).  The chunk's reflectors go back into the panel; its R, tau and the
// compact-WY factor T (w x w upper triangular, Q = H_0 ... H_{w-1} = I - V T V^T,
// dlarft forward/columnwise) go into the tree storage.  R factors are then merged
// pairwise up a binary tree by QR of the stacked [R_left; R_right] (2w x w); the
// work-group that finishes second on a pair performs the merge (an atomic counter
// per node, reset by that group), so the whole tree runs in one launch and no
// group waits on another.  An odd last node is merged with a zero sibling, which
// gives tau = 0 (identity).
//
// Apply: out = Q [X; 0] for the explicit thin factor Q (h x w).  Each chunk's
// group walks from the root to its chunk; at every node [X; 0] - V (T (V_top^T X))
// gives the node's 2w rows, of which the half belonging to the child is kept;
// at the chunk the same three small products give the output rows.  Optionally
// adds U1 * Tm (the merge's U1 U_E,top term).
#include "hsvd_internal.hpp"
#include "device_common.hpp"
#include "house_qr.hpp"

namespace hsvd {

constexpr int TSQR_THREADS = 1024;

// Node slot layout: R (w*w) | V (2w*w) | tau (w) | T (w*w)
__device__ __forceinline__ int64_t slot_tau(int w) { return 3LL * w * w; }
__device__ __forceinline__ int64_t slot_T(int w) { return 3LL * w * w + w; }

// Slot index of tree node (level, idx) given the chunk count.
__device__ __forceinline__ int node_slot(int nch, int level, int idx) {
    int off = 0, n = nch;
    for (int l = 0; l < level; ++l) { off += n; n = (n + 1) >> 1; }
    return off + idx;
}

// Element (i, l) of the reflector block V whose strictly-lower part is stored in
// the column-major array A (ld) with the unit diagonal implicit.
__device__ __forceinline__ double vref(const double* A, int64_t ld, int i, int l) {
    return i == l ? 1.0 : (i > l ? A[(int64_t)l * ld + i] : 0.0);
}

// MT: registers live in a tree merge (2w <= LANES * MT rows)
template <int LANES, int RMAX, int MT>
__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr_factor(double* __restrict__ ws,
                                                              int* __restrict__ iws,
                                                              const TsqrTask* __restrict__ tasks,
                                                              const ChunkRef* __restrict__ chunks,
                                                              int w, int ch) {
    extern __shared__ double sm[];
    double* T = sm;                                  // w x (w + 1)
    double* tau = T + (int64_t)w * (w + 1);
    double* z = tau + w;                             // 2w
    double* vbuf = z + 2 * w;                        // 2 * LANES * RMAX
    __shared__ int s_go;
    HouseQR<LANES, RMAX> q;

    const ChunkRef cr = chunks[blockIdx.x];
    const TsqrTask t = tasks[cr.task];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    double* P = ws + t.p_off;
    double* store = ws + t.store_off;
    const int64_t S = tsqr_slot_size(w);

    q.load(P + row0, t.p_ld, rows, w);
    q.factor(rows, w, T, tau, z, vbuf);
    q.store(P + row0, t.p_ld, rows, w);
    {
        double* slot = store + S * node_slot(t.nch, 0, cr.chunk);
        q.store_r(slot, rows, w);
        for (int e = tid; e < w * w; e += nth) {
            const int j = e / w, i = e - j * w;
            slot[slot_T(w) + e] = T[(int64_t)j * (w + 1) + i];
        }
        for (int j = tid; j < w; j += nth) slot[slot_tau(w) + j] = tau[j];
    }
    int level = 0, idx = cr.chunk, n = t.nch;
    int last_rows = rows;
    while (n > 1) {
        const int parent = idx >> 1;
        const bool has_sib = ((idx ^ 1) < n);
        __threadfence();
        __syncthreads();
        if (has_sib) {
            if (tid == 0) {
                const int slot = node_slot(t.nch, level + 1, parent);
                const int old = atomicAdd(&iws[t.cnt_off + slot], 1);
                s_go = (old == 1);
                if (old == 1) atomicExch(&iws[t.cnt_off + slot], 0);
            }
            __syncthreads();
            if (!s_go) return;
        }
        __threadfence();
        // stack [R_left; R_right (or 0)] -> 2w x w, straight into registers
        const int left = parent * 2;
        const double* Rl = store + S * node_slot(t.nch, level, left);
        const double* Rr = has_sib ? store + S * node_slot(t.nch, level, left + 1) : nullptr;
        {
            const int c = tid / LANES, gl = tid % LANES;
#pragma unroll
            for (int tt = 0; tt < RMAX; ++tt) {
                const int r = gl + LANES * tt;
                double v = 0.0;
                if (c < w && r < 2 * w) {
                    if (r < w) v = Rl[(int64_t)c * w + r];
                    else if (Rr) v = Rr[(int64_t)c * w + (r - w)];
                }
                q.x[tt] = v;
            }
        }
        // the stacked pair has 2w rows: only the first MT registers are live
        q.template factor<MT>(2 * w, w, T, tau, z, vbuf);
        double* slot = store + S * node_slot(t.nch, level + 1, parent);
        q.store_r(slot, 2 * w, w);
        q.store(slot + w * w, 2 * w, 2 * w, w);
        for (int e = tid; e < w * w; e += nth) {
            const int j = e / w, i = e - j * w;
            slot[slot_T(w) + e] = T[(int64_t)j * (w + 1) + i];
        }
        for (int j = tid; j < w; j += nth) slot[slot_tau(w) + j] = tau[j];
        last_rows = 2 * w;
        ++level;
        idx = parent;
        n = (n + 1) >> 1;
    }
    q.store_r(ws + t.r_out, last_rows, w);
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

// One compact-WY level on LDS operands: W1 = V_top^T X (V_top staged in Vs, ld w),
// then W2 = T W1 (T from global, col-major ld w) written back over W1
// (w * c <= 8 * blockDim.x).
__device__ void wy_w(const double* Vs, const double* Tg, const double* X, double* W, int w, int c) {
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int e = tid; e < w * c; e += nth) {
        const int cc = e / w, l = e - cc * w;
        double d = 0.0;
        for (int i = l; i < w; ++i) d = fma(Vs[(int64_t)l * w + i], X[(int64_t)cc * w + i], d);
        W[e] = d;
    }
    __syncthreads();
    double r[8];
    int cnt = 0;
    for (int e = tid; e < w * c; e += nth, ++cnt) {
        const int cc = e / w, i = e - cc * w;
        double d = 0.0;
        for (int l = i; l < w; ++l) d = fma(Tg[(int64_t)l * w + i], W[(int64_t)cc * w + l], d);
        r[cnt] = d;
    }
    __syncthreads();
    cnt = 0;
    for (int e = tid; e < w * c; e += nth, ++cnt) W[e] = r[cnt];
    __syncthreads();
}

__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr_apply(double* __restrict__ ws,
                                                             const TsqrTask* __restrict__ tsqr,
                                                             const ApplyTask* __restrict__ tasks,
                                                             const ChunkRef* __restrict__ chunks,
                                                             int w, int ch, int c) {
    extern __shared__ double sm[];
    double* X = sm;                                  // w x c (ld w)
    double* W = X + (int64_t)w * c;                  // w x c
    double* Vs = W + (int64_t)w * c;                 // w x w staged reflector rows
    const ChunkRef cr = chunks[blockIdx.x];
    const ApplyTask a = tasks[cr.task];
    const TsqrTask t = tsqr[a.tsqr];
    const int tid = threadIdx.x, nth = blockDim.x;
    const double* store = ws + t.store_off;
    const int64_t S = tsqr_slot_size(w);

    const double* Xg = ws + a.x_off;
    for (int e = tid; e < w * c; e += nth) X[e] = Xg[e];
    int levels = 0;
    for (int n = t.nch; n > 1; n = (n + 1) >> 1) ++levels;
    for (int level = levels; level >= 1; --level) {
        const int idx = cr.chunk >> level;
        const bool right = (cr.chunk >> (level - 1)) & 1;
        const double* slot = store + S * node_slot(t.nch, level, idx);
        const double* V = slot + w * w;              // 2w x w, ld 2w
        stage_v(V, 2 * w, 0, w, w, Vs, w);
        __syncthreads();
        wy_w(Vs, slot + slot_T(w), X, W, w, c);
        if (right) {
            stage_v(V, 2 * w, w, w, w, Vs, w);
            __syncthreads();
        }
        for (int e = tid; e < w * c; e += nth) {
            const int cc = e / w, i = e - cc * w;
            double d = right ? 0.0 : X[e];
            for (int l = 0; l < w; ++l) d = fma(-Vs[(int64_t)l * w + i], W[(int64_t)cc * w + l], d);
            X[e] = d;                                  // each entry reads only itself from X
        }
        __syncthreads();
    }
    // chunk level: out = [X; 0] - V (T (V_top^T X)) over the chunk rows
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    const double* Vc = ws + t.p_off + row0;
    const double* cslot = store + S * node_slot(t.nch, 0, cr.chunk);
    const int vtop = rows < w ? rows : w;
    stage_v(Vc, t.p_ld, 0, vtop, w, Vs, w);
    for (int e = tid; e < (w - vtop) * w; e += nth) {     // rows past a short chunk: zero
        const int l = e / (w - vtop), i = vtop + e - l * (w - vtop);
        Vs[(int64_t)l * w + i] = 0.0;
    }
    __syncthreads();
    wy_w(Vs, cslot + slot_T(w), X, W, w, c);
    double* out = ws + a.out_off;
    const double* U1 = a.add_u_off >= 0 ? ws + a.add_u_off : nullptr;
    const double* Tm = a.add_u_off >= 0 ? ws + a.add_t_off : nullptr;
    for (int r0 = 0; r0 < rows; r0 += w) {
        const int nrow = min(w, rows - r0);
        if (r0 > 0) {
            __syncthreads();
            stage_v(Vc, t.p_ld, r0, nrow, w, Vs, w);
            __syncthreads();
        }
        for (int e = tid; e < nrow * c; e += nth) {
            const int cc = e / nrow, ii = e - cc * nrow;
            const int i = r0 + ii;
            double d = (i < w) ? X[(int64_t)cc * w + i] : 0.0;
            for (int l = 0; l < w; ++l) d = fma(-Vs[(int64_t)l * w + ii], W[(int64_t)cc * w + l], d);
            if (U1)
                for (int l = 0; l < a.add_w; ++l)
                    d = fma(U1[(int64_t)l * a.add_u_ld + row0 + i], Tm[(int64_t)cc * a.add_w + l], d);
            out[(int64_t)cc * a.out_ld + row0 + i] = d;
        }
    }
}

template <int LANES, int RMAX, int MT>
static hipError_t launch_factor_t(double* ws, int* iws, const TsqrTask* tasks,
                                  const ChunkRef* chunks, int nchunks, int w, int ch, hipStream_t s) {
    const size_t lds = sizeof(double) * (HouseQR<LANES, RMAX>::lds_doubles(w) + 32);
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_factor<LANES, RMAX, MT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tsqr_factor<LANES, RMAX, MT>), dim3(nchunks), dim3(TSQR_THREADS), lds, s, ws,
                       iws, tasks, chunks, w, ch);
    return hipGetLastError();
}

hipError_t launch_tsqr_factor(double* ws, int* iws, const TsqrTask* tasks, const ChunkRef* chunks,
                              int nchunks, int w, int ch, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    if (w < 1 || w > kTsqrMaxW || ch != tsqr_chunk_rows(w)) return hipErrorInvalidValue;
    // a chunk and a stacked pair of R factors must fit the register block
    if (w <= 64) {
        if (ch > 16 * 16 || 2 * w > 16 * 8) return hipErrorInvalidValue;
        return launch_factor_t<16, 16, 8>(ws, iws, tasks, chunks, nchunks, w, ch, s);
    }
    if (ch > 8 * 20 || 2 * w > 8 * 20) return hipErrorInvalidValue;
    return launch_factor_t<8, 20, 20>(ws, iws, tasks, chunks, nchunks, w, ch, s);
}

hipError_t launch_tsqr_apply(double* ws, const TsqrTask* tsqr, const ApplyTask* tasks,
                             const ChunkRef* chunks, int nchunks, int w, int ch, int c,
                             hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (2 * (size_t)w * c + (size_t)w * w + 32);
    if (w * c > 8 * TSQR_THREADS) return hipErrorInvalidValue;   // wy_w keeps 8 values per thread
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tsqr_apply, dim3(nchunks), dim3(TSQR_THREADS), lds, s, ws, tsqr, tasks,
                       chunks, w, ch, c);
    return hipGetLastError();
}

}  // namespace hsvd
