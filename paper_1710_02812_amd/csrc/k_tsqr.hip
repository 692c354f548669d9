// Tall-skinny Householder QR (TSQR) for h x w panels, w <= 96.
//
// Factor: each row chunk of `ch` rows is loaded into LDS and reduced by w
// Householder reflectors (LAPACK dlarfg convention: H = I - tau v v^T, v_j = 1,
// R_jj = beta).  The chunk's reflectors go back into the panel and its R into the
// tree storage.  R factors are then merged pairwise up a binary tree by QR of the
// stacked [R_left; R_right] (2w x w); the work-group that finishes second on a
// pair performs the merge (an atomic counter per node, reset by that group), so
// the whole tree runs in one launch without any group waiting on another.  An
// odd last node is "merged" with a zero sibling, which yields tau = 0 (identity).
//
// Apply: out = Q [X; 0] for the explicit thin factor Q (h x w).  Each chunk's
// group walks from the root to its chunk, applying every node's reflectors to
// [X; 0] and keeping the half that belongs to its child, then applies the chunk
// reflectors.  Optionally adds U1 * T (the merge's U1 U_E,top term).
#include "hsvd_internal.hpp"
#include "device_common.hpp"

namespace hsvd {

constexpr int TSQR_THREADS = 256;

__device__ __forceinline__ int64_t node_slot_size(int w) { return 3LL * w * w + w; }

// Slot index of tree node (level, idx) given the chunk count.
__device__ __forceinline__ int node_slot(int nch, int level, int idx) {
    int off = 0, n = nch;
    for (int l = 0; l < level; ++l) { off += n; n = (n + 1) >> 1; }
    return off + idx;
}

// Householder QR of the rows x w matrix in LDS (column stride lds), in place.
__device__ void house_qr_lds(double* A, int lds, int rows, int w, double* tau, double* red) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    const int kmax = rows < w ? rows : w;
    for (int j = 0; j < kmax; ++j) {
        double* aj = A + (int64_t)j * lds;
        double s = 0.0;
        for (int i = j + 1 + tid; i < rows; i += nth) s += aj[i] * aj[i];
        s = block_sum(s, red);
        const double alpha = aj[j];
        double beta = alpha, tj = 0.0, scal = 0.0;
        if (s > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + s), alpha);
            tj = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        __syncthreads();
        if (s > 0.0)
            for (int i = j + 1 + tid; i < rows; i += nth) aj[i] *= scal;
        if (tid == 0) { aj[j] = beta; tau[j] = tj; }
        __syncthreads();
        if (tj != 0.0) {
            for (int c = j + 1 + wave; c < w; c += nw) {
                double* ac = A + (int64_t)c * lds;
                double d = (lane == 0) ? ac[j] : 0.0;
                for (int i = j + 1 + lane; i < rows; i += 64) d += aj[i] * ac[i];
                d = wave_sum(d);
                const double f = tj * d;
                if (lane == 0) ac[j] -= f;
                for (int i = j + 1 + lane; i < rows; i += 64) ac[i] -= f * aj[i];
            }
        }
        __syncthreads();
    }
    for (int j = kmax + tid; j < w; j += nth) tau[j] = 0.0;
    __syncthreads();
}

// Y (rows x c in LDS, stride ldy) <- H_0 ... H_{w-1} Y with reflectors v_j taken from
// `V` (column j at V + j*ldv, rows j+1.. below the implicit unit) and tau.
// `V` may be global or LDS memory.
__device__ void apply_q_lds(const double* V, int64_t ldv, const double* tau, int rows, int w,
                            double* Y, int ldy, int c) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int kmax = rows < w ? rows : w;
    for (int j = kmax - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;                    // uniform across the group
        const double* vj = V + (int64_t)j * ldv;
        for (int cc = wave; cc < c; cc += nw) {
            double* yc = Y + (int64_t)cc * ldy;
            double d = (lane == 0) ? yc[j] : 0.0;
            for (int i = j + 1 + lane; i < rows; i += 64) d += vj[i] * yc[i];
            d = wave_sum(d);
            const double f = tj * d;
            if (lane == 0) yc[j] -= f;
            for (int i = j + 1 + lane; i < rows; i += 64) yc[i] -= f * vj[i];
        }
        __syncthreads();
    }
    __syncthreads();
}

__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr_factor(double* __restrict__ ws,
                                                              int* __restrict__ iws,
                                                              const TsqrTask* __restrict__ tasks,
                                                              const ChunkRef* __restrict__ chunks,
                                                              int w, int ch) {
    extern __shared__ double sm[];
    const int lds = (ch > 2 * w ? ch : 2 * w) + 1;
    double* A = sm;
    double* tau = A + (int64_t)w * lds;
    double* red = tau + w + 1;
    __shared__ int s_go;

    const ChunkRef cr = chunks[blockIdx.x];
    const TsqrTask t = tasks[cr.task];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    double* P = ws + t.p_off;
    double* store = ws + t.store_off;
    const int64_t S = node_slot_size(w);

    for (int e = tid; e < rows * w; e += nth) {
        const int j = e / rows, i = e - j * rows;
        A[(int64_t)j * lds + i] = P[(int64_t)j * t.p_ld + row0 + i];
    }
    __syncthreads();
    house_qr_lds(A, lds, rows, w, tau, red);

    // chunk reflectors back into the panel, R and tau into the node slot
    for (int e = tid; e < rows * w; e += nth) {
        const int j = e / rows, i = e - j * rows;
        P[(int64_t)j * t.p_ld + row0 + i] = A[(int64_t)j * lds + i];
    }
    {
        double* slot = store + S * node_slot(t.nch, 0, cr.chunk);
        for (int e = tid; e < w * w; e += nth) {
            const int j = e / w, i = e - j * w;
            slot[e] = (i <= j && i < rows) ? A[(int64_t)j * lds + i] : 0.0;
        }
        for (int j = tid; j < w; j += nth) slot[3 * w * w + j] = tau[j];
    }

    int level = 0, idx = cr.chunk, n = t.nch;
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
        // stack [R_left; R_right (or 0)] -> 2w x w
        const int left = parent * 2, right = left + 1;
        const double* Rl = store + S * node_slot(t.nch, level, left);
        const double* Rr = has_sib ? store + S * node_slot(t.nch, level, right) : nullptr;
        for (int e = tid; e < 2 * w * w; e += nth) {
            const int j = e / (2 * w), i = e - j * (2 * w);
            double v;
            if (i < w) v = Rl[(int64_t)j * w + i];
            else v = Rr ? Rr[(int64_t)j * w + (i - w)] : 0.0;
            A[(int64_t)j * lds + i] = v;
        }
        __syncthreads();
        house_qr_lds(A, lds, 2 * w, w, tau, red);
        double* slot = store + S * node_slot(t.nch, level + 1, parent);
        for (int e = tid; e < w * w; e += nth) {
            const int j = e / w, i = e - j * w;
            slot[e] = (i <= j) ? A[(int64_t)j * lds + i] : 0.0;
        }
        for (int e = tid; e < 2 * w * w; e += nth) {
            const int j = e / (2 * w), i = e - j * (2 * w);
            slot[w * w + e] = A[(int64_t)j * lds + i];
        }
        for (int j = tid; j < w; j += nth) slot[3 * w * w + j] = tau[j];
        ++level;
        idx = parent;
        n = (n + 1) >> 1;
    }
    // root: its factorisation is the last one this group ran, still in LDS
    double* R = ws + t.r_out;
    const int rr = (t.nch == 1) ? rows : 2 * w;
    for (int e = tid; e < w * w; e += nth) {
        const int j = e / w, i = e - j * w;
        R[e] = (i <= j && i < rr) ? A[(int64_t)j * lds + i] : 0.0;
    }
}

__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr_apply(double* __restrict__ ws,
                                                             const TsqrTask* __restrict__ tsqr,
                                                             const ApplyTask* __restrict__ tasks,
                                                             const ChunkRef* __restrict__ chunks,
                                                             int w, int ch, int c) {
    extern __shared__ double sm[];
    const int ldy = (ch > 2 * w ? ch : 2 * w) + 1;
    double* Y = sm;                                  // ldy x c
    double* taus = Y + (int64_t)c * ldy;             // w
    const ChunkRef cr = chunks[blockIdx.x];
    const ApplyTask a = tasks[cr.task];
    const TsqrTask t = tsqr[a.tsqr];
    const int tid = threadIdx.x, nth = blockDim.x;
    const double* store = ws + t.store_off;
    const int64_t S = node_slot_size(w);

    // X -> top of Y
    const double* X = ws + a.x_off;
    for (int e = tid; e < w * c; e += nth) {
        const int j = e / w, i = e - j * w;
        Y[(int64_t)j * ldy + i] = X[(int64_t)j * w + i];
    }
    // levels: count
    int levels = 0;
    for (int n = t.nch; n > 1; n = (n + 1) >> 1) ++levels;
    for (int level = levels; level >= 1; --level) {
        const int idx = cr.chunk >> level;
        const int child = cr.chunk >> (level - 1);
        const double* slot = store + S * node_slot(t.nch, level, idx);
        for (int e = tid; e < w * c; e += nth) {
            const int j = e / w, i = e - j * w;
            Y[(int64_t)j * ldy + w + i] = 0.0;
        }
        for (int j = tid; j < w; j += nth) taus[j] = slot[3 * w * w + j];
        __syncthreads();
        apply_q_lds(slot + w * w, 2 * w, taus, 2 * w, w, Y, ldy, c);
        if (child & 1) {   // keep the bottom half
            for (int e = tid; e < w * c; e += nth) {   // disjoint rows: no hazard
                const int j = e / w, i = e - j * w;
                Y[(int64_t)j * ldy + i] = Y[(int64_t)j * ldy + w + i];
            }
        }
        __syncthreads();
    }
    // chunk level
    const int row0 = cr.chunk * ch;
    const int rows = min(ch, t.h - row0);
    for (int e = tid; e < (rows - w > 0 ? rows - w : 0) * c; e += nth) {
        const int span = rows - w;
        const int j = e / span, i = e - j * span;
        Y[(int64_t)j * ldy + w + i] = 0.0;
    }
    {
        const double* cslot = store + S * node_slot(t.nch, 0, cr.chunk);
        for (int j = tid; j < w; j += nth) taus[j] = cslot[3 * w * w + j];
    }
    __syncthreads();
    const double* Vc = ws + t.p_off + row0;
    apply_q_lds(Vc, t.p_ld, taus, rows, w, Y, ldy, c);
    __syncthreads();
    double* out = ws + a.out_off;
    if (a.add_u_off >= 0) {
        const double* U1 = ws + a.add_u_off;
        const double* T = ws + a.add_t_off;
        for (int e = tid; e < rows * c; e += nth) {
            const int j = e / rows, i = e - j * rows;
            double v = Y[(int64_t)j * ldy + i];
            for (int l = 0; l < a.add_w; ++l)
                v = fma(U1[(int64_t)l * a.add_u_ld + row0 + i], T[(int64_t)j * a.add_w + l], v);
            out[(int64_t)j * a.out_ld + row0 + i] = v;
        }
    } else {
        for (int e = tid; e < rows * c; e += nth) {
            const int j = e / rows, i = e - j * rows;
            out[(int64_t)j * a.out_ld + row0 + i] = Y[(int64_t)j * ldy + i];
        }
    }
}

static size_t tsqr_lds_bytes(int w, int ch, int c) {
    const int ld = (ch > 2 * w ? ch : 2 * w) + 1;
    const int cols = c > w ? c : w;
    return sizeof(double) * ((size_t)cols * ld + w + 1 + 16);
}

hipError_t launch_tsqr_factor(double* ws, int* iws, const TsqrTask* tasks, const ChunkRef* chunks,
                              int nchunks, int w, int ch, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = tsqr_lds_bytes(w, ch, w);
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_factor,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tsqr_factor, dim3(nchunks), dim3(TSQR_THREADS), lds, s, ws, iws, tasks,
                       chunks, w, ch);
    return hipGetLastError();
}

hipError_t launch_tsqr_apply(double* ws, const TsqrTask* tsqr, const ApplyTask* tasks,
                             const ChunkRef* chunks, int nchunks, int w, int ch, int c,
                             hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = tsqr_lds_bytes(w, ch, c);
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tsqr_apply, dim3(nchunks), dim3(TSQR_THREADS), lds, s, ws, tsqr, tasks,
                       chunks, w, ch, c);
    return hipGetLastError();
}

}  // namespace hsvd
