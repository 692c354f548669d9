// Kernel-level entry points (hsvd_debug.h): run the Jacobi core or the TSQR
// factor/apply kernels on caller data, with a private scratch arena.
#include "../../include/hsvd_debug.h"
#include "hsvd_internal.hpp"

#include <algorithm>
#include <string>
#include <vector>

using namespace hsvd;

extern "C" const char* hsvd_last_error(void);
namespace hsvd_detail {
hsvd_status set_error(hsvd_status st, const std::string& msg);
}

namespace {

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) hipFree(p);
    }
    template <typename T>
    T* get(size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T*)p;
    }
};

int pow2floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

}  // namespace

extern "C" hsvd_status hsvd_debug_jacobi(const double* M, int32_t batch, int32_t n, double* U,
                                         double* S, double* V, int32_t max_sweeps,
                                         int32_t precondition, uint32_t* flags_host,
                                         hipStream_t stream) {
    using hsvd_detail::set_error;
    if (!M || !U || !S || batch < 1 || n < 1 || n > kWideCoreMaxN || (V && n > kCoreMaxV) || max_sweeps < 1 ||
        (precondition != 0 && precondition != 1) || (precondition && V))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_jacobi: bad argument");
    Scratch sc;
    const int64_t nn = (int64_t)n * n;
    const bool wide = n > kCoreMaxN;
    // arena: copies of M | U | V | S | wide-core scratch panels
    const int64_t offM = 0, offU = offM + batch * nn, offV = offU + batch * nn,
                  offS = offV + batch * nn, offW = offS + (int64_t)batch * n,
                  tot = offW + (wide ? batch * kWideScratch : 0);
    double* ws = sc.get<double>(tot);
    int* iws = sc.get<int>(batch);
    unsigned* flags = sc.get<unsigned>(2);
    CoreTask* dt = sc.get<CoreTask>(batch);
    if (!ws || !iws || !flags || !dt) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    std::vector<CoreTask> tasks(batch);
    for (int b = 0; b < batch; ++b) {
        CoreTask c{};
        c.mode = CORE_DENSE;
        c.dim = n;
        c.m_off = offM + b * nn;
        c.m_ld = n;
        c.rank_in = -1;
        c.rank1 = c.rank2 = -1;
        c.u_off = offU + b * nn;
        c.u_ld = n;
        c.t_off = -1;
        c.v_off = V ? offV + b * nn : -1;
        c.v_ld = n;
        c.sig_off = offS + (int64_t)b * n;
        c.out_w = n;
        c.rank_out = b;
        c.kcap = n;
        c.rule = 0;
        c.tol = 0.0;
        c.floor_rows = 0;
        c.floor_cols = -1;
        c.fixed_rank_slot = -1;
        c.precond = precondition;
        c.scr_off = wide ? offW + b * kWideScratch : -1;
        c.energy_off = -1;
        c.flag_slot = -1;
        // keep every nonzero column: rank = count above a zero floor of 0
        tasks[b] = c;
    }
    hipError_t e = hipMemcpyAsync(ws + offM, M, sizeof(double) * batch * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tasks.data(), sizeof(CoreTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(flags, 0, 2 * sizeof(unsigned), stream);
    if (e == hipSuccess) e = launch_core(ws, iws, dt, batch, n, max_sweeps, flags, V ? 1 : 0, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(U, ws + offU, sizeof(double) * batch * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(S, ws + offS, sizeof(double) * batch * n, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && V) e = hipMemcpyAsync(V, ws + offV, sizeof(double) * batch * nn, hipMemcpyDeviceToDevice, stream);
    unsigned fl[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(fl, flags, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_jacobi: ") + hipGetErrorString(e));
    if (flags_host) *flags_host = (fl[0] & 0xFFFFu) | (std::min(fl[1], 0xFFFFu) << 16);
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_debug_gemm(int32_t op, int32_t kind, int32_t a_fp32, const void* A,
                                       int64_t rows, int64_t cols, int64_t lda, const double* X,
                                       int32_t N, double* Y, hipStream_t stream) {
    using hsvd_detail::set_error;
    if (!A || !X || !Y || (op != 0 && op != 1) || kind < 0 || kind > 2 || rows < 1 || cols < 1 ||
        lda < cols || N < 1 || N > 1024 || (kind != 0 && !a_fp32) || rows > (1 << 20) || cols > (1 << 20))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_gemm: bad argument");
    const int64_t xr = op == 0 ? cols : rows, yr = op == 0 ? rows : cols;
    Scratch sc;
    double* ws = sc.get<double>(xr * N + yr * N);
    GemmTask* dt = sc.get<GemmTask>(1);
    void** dptrs = sc.get<void*>(4);
    const int tile_rows = kind != 0 ? kBf16TileRows : 64;
    if (kind != 0 && N > kBf16MaxN)
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_gemm: bfloat16 and float32 passes take N <= 96");
    const int nrt = (int)((yr + tile_rows - 1) / tile_rows), nct = kind != 0 ? 1 : gemm_f64_col_tiles(N);
    TileRef* dtiles = sc.get<TileRef>((size_t)nrt * nct);
    if (!ws || !dt || !dtiles || !dptrs) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    GemmTask t{};
    t.a_off = 0;
    t.lda = lda;
    t.mat = 0;
    t.x_off = 0;
    t.y_off = xr * N;
    t.rows = (int32_t)rows;
    t.cols = (int32_t)cols;
    t.x_ld = (int32_t)xr;
    t.y_ld = (int32_t)yr;
    t.tiles = nrt;
    std::vector<TileRef> tiles((size_t)nrt * nct);
    for (int i = 0; i < nrt * nct; ++i) tiles[i] = {0, i};
    void* tab[4] = {const_cast<void*>(A), nullptr, nullptr, nullptr};
    hipError_t e = hipMemcpyAsync(ws, X, sizeof(double) * xr * N, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dptrs, tab, sizeof(tab), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, &t, sizeof(t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dtiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = kind == 1   ? launch_gemm_bf16(op, (const void* const*)dptrs, ws, dt, dtiles, nrt * nct, N, stream)
            : kind == 2 ? launch_gemm_f32(op, (const void* const*)dptrs, ws, dt, dtiles, nrt * nct, N, stream)
                        : launch_gemm(op, a_fp32, (const void* const*)dptrs, ws, dt, dtiles, nrt * nct, N, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Y, ws + xr * N, sizeof(double) * yr * N, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_gemm: ") + hipGetErrorString(e));
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_debug_tsqr(const double* P, int32_t batch, int64_t h, int32_t w,
                                       double* Q, double* R, hipStream_t stream) {
    using hsvd_detail::set_error;
    if (!P || !Q || !R || batch < 1 || h < 1 || w < 1 || w > kTsqrMaxW || h > (1 << 26))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_tsqr: bad argument");
    Scratch sc;
    const int ch = tsqr_chunk_rows(w);
    const int nch = (int)((h + ch - 1) / ch);
    const int nodes = tsqr_nodes(nch, tsqr_fanin(w));
    const int64_t hw = h * w, slot = tsqr_slot_size(w);
    const int64_t offP = 0, offI = offP + batch * hw, offQ = offI + (int64_t)w * w,
                  offS = offQ + batch * hw, offR = offS + (int64_t)batch * nodes * slot,
                  tot = offR + (int64_t)batch * w * w;
    double* ws = sc.get<double>(tot);
    int* iws = sc.get<int>((size_t)batch * nodes);
    TsqrTask* dt = sc.get<TsqrTask>(batch);
    ApplyTask* da = sc.get<ApplyTask>(batch);
    ChunkRef* dc = sc.get<ChunkRef>((size_t)batch * nch);
    if (!ws || !iws || !dt || !da || !dc) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    std::vector<TsqrTask> tt(batch);
    std::vector<ApplyTask> at(batch);
    std::vector<ChunkRef> cr;
    for (int b = 0; b < batch; ++b) {
        TsqrTask t{};
        t.p_off = offP + b * hw;
        t.store_off = offS + (int64_t)b * nodes * slot;
        t.r_out = offR + (int64_t)b * w * w;
        t.h = (int)h;
        t.p_ld = (int)h;
        t.nch = nch;
        t.chunk0 = b * nch;
        t.cnt_off = b * nodes;
        t.levels = tsqr_levels(nch, tsqr_fanin(w));
        tt[b] = t;
        ApplyTask a{};
        a.tsqr = b;
        a.x_off = offI;
        a.out_off = offQ + b * hw;
        a.out_ld = (int)h;
        a.add_u_off = -1;
        at[b] = a;
        for (int c = 0; c < nch; ++c) cr.push_back({b, c});
    }
    std::vector<double> I((size_t)w * w, 0.0);
    for (int i = 0; i < w; ++i) I[(size_t)i * w + i] = 1.0;
    hipError_t e = hipMemcpyAsync(ws + offP, P, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + offI, I.data(), sizeof(double) * w * w, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(iws, 0, sizeof(int) * batch * nodes, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tt.data(), sizeof(TsqrTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(da, at.data(), sizeof(ApplyTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, cr.data(), sizeof(ChunkRef) * cr.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_tsqr_factor(ws, iws, dt, dc, (int)cr.size(), w, ch, stream);
    if (e == hipSuccess) e = launch_tsqr_apply(ws, iws, dt, da, dc, (int)cr.size(), w, ch, w, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Q, ws + offQ, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(R, ws + offR, sizeof(double) * batch * w * w, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_tsqr: ") + hipGetErrorString(e));
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_debug_cholqr(const double* P, int32_t batch, int64_t h, int32_t w, double* Q,
                                         double* R, int32_t* fell_back, hipStream_t stream) {
    using hsvd_detail::set_error;
    if (!P || !Q || !R || !fell_back || batch < 1 || h < 1 || w < 1 || w > 64 || h > (1 << 26))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_cholqr: bad argument");
    Scratch sc;
    const int ch = tsqr_chunk_rows(w);
    const int nch = (int)((h + ch - 1) / ch);
    const int nodes = tsqr_nodes(nch, tsqr_fanin(w));
    const int cnodes = std::max(1, cq_nodes(nch));
    const int nthin = (int)((h + THIN_CH - 1) / THIN_CH);
    const int64_t hw = h * w, ww = (int64_t)w * w, slot = tsqr_slot_size(w), cqs = cq_size(w, nch, (int)h);
    const int64_t offP = 0, offI = offP + batch * hw, offQ = offI + ww, offS = offQ + batch * hw,
                  offR = offS + (int64_t)batch * nodes * slot, offCQ = offR + batch * ww,
                  offC = offCQ + batch * cqs, tot = offC + batch * ww;
    const int iper = nodes + 1 + cnodes;
    double* ws = sc.get<double>(tot);
    int* iws = sc.get<int>((size_t)batch * iper);
    TsqrTask* dt = sc.get<TsqrTask>(batch);
    ApplyTask* da = sc.get<ApplyTask>(batch);
    ChunkRef* dc = sc.get<ChunkRef>((size_t)batch * nch);
    ThinTask* dn = sc.get<ThinTask>(3 * (size_t)batch);
    ChunkRef* dnc = sc.get<ChunkRef>((size_t)batch * (2 * nthin + 1));
    if (!ws || !iws || !dt || !da || !dc || !dn || !dnc) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    std::vector<TsqrTask> tt(batch);
    std::vector<ApplyTask> at(batch);
    std::vector<ThinTask> nn(3 * (size_t)batch);           // Q1 = P M1 | C = M2 I | Q = Q1 C
    std::vector<ChunkRef> cr, ncr;
    for (int b = 0; b < batch; ++b) {
        TsqrTask t{};
        t.p_off = offP + b * hw;
        t.store_off = offS + (int64_t)b * nodes * slot;
        t.r_out = offR + b * ww;
        t.h = (int)h;
        t.p_ld = (int)h;
        t.nch = nch;
        t.chunk0 = b * nch;
        t.cnt_off = b * iper;
        t.levels = tsqr_levels(nch, tsqr_fanin(w));
        t.cq_off = offCQ + b * cqs;
        t.cq_flag = b * iper + nodes;
        t.cq_cnt = t.cq_flag + 1;
        tt[b] = t;
        ApplyTask a{};
        a.tsqr = b;
        a.x_off = offI;
        a.out_off = offQ + b * hw;
        a.out_ld = (int)h;
        a.add_u_off = -1;
        at[b] = a;
        for (int c = 0; c < nch; ++c) cr.push_back({b, c});
        ThinTask& x = nn[b];                                // Q1 = P M1
        x.x_off = t.p_off; x.x_ld = (int)h;
        x.c_off = t.cq_off + ww; x.c_ld = w;
        x.y_off = t.cq_off + cq_q1(w, nch); x.y_ld = (int)h;
        x.h = (int)h; x.wx = w; x.wy = w; x.cond = t.cq_flag;
        ThinTask& y = nn[batch + b];                        // C = M2 I
        y.x_off = t.cq_off + 2 * ww; y.x_ld = w;
        y.c_off = offI; y.c_ld = w;
        y.y_off = offC + b * ww; y.y_ld = w;
        y.h = w; y.wx = w; y.wy = w; y.cond = t.cq_flag;
        ThinTask& z = nn[2 * batch + b];                    // Q = Q1 C
        z.x_off = x.y_off; z.x_ld = (int)h;
        z.c_off = y.y_off; z.c_ld = w;
        z.y_off = a.out_off; z.y_ld = (int)h;
        z.h = (int)h; z.wx = w; z.wy = w; z.cond = t.cq_flag;
    }
    // chunk lists of the three products: [Q1 | C | Q], each task's chunks in order
    int n0 = 0, n1 = 0, n2 = 0;
    for (int part = 0; part < 3; ++part)
        for (int b = 0; b < batch; ++b) {
            ThinTask& x = nn[part * batch + b];
            x.nch = (x.h + THIN_CH - 1) / THIN_CH;
            x.chunk0 = (int)ncr.size();
            for (int c = 0; c < x.nch; ++c) ncr.push_back({b, c});
            (part == 0 ? n0 : part == 1 ? n1 : n2) += x.nch;
        }
    for (int part = 0; part < 3; ++part)
        for (int b = 0; b < batch; ++b) nn[part * batch + b].chunk0 -= (part == 0 ? 0 : part == 1 ? n0 : n0 + n1);
    std::vector<double> I((size_t)ww, 0.0);
    for (int i = 0; i < w; ++i) I[(size_t)i * w + i] = 1.0;
    hipError_t e = hipMemcpyAsync(ws + offP, P, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + offI, I.data(), sizeof(double) * ww, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(iws, 0, sizeof(int) * batch * iper, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tt.data(), sizeof(TsqrTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(da, at.data(), sizeof(ApplyTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, cr.data(), sizeof(ChunkRef) * cr.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dn, nn.data(), sizeof(ThinTask) * nn.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dnc, ncr.data(), sizeof(ChunkRef) * ncr.size(), hipMemcpyHostToDevice, stream);
    const int nc = (int)cr.size();
    if (e == hipSuccess) e = launch_cholqr(1, ws, iws, dt, dc, nc, w, ch, stream);
    if (e == hipSuccess) e = launch_thin_nn(ws, iws, dn, dnc, n0, THIN_CH, stream);
    if (e == hipSuccess) e = launch_cholqr(2, ws, iws, dt, dc, nc, w, ch, stream);
    if (e == hipSuccess) e = launch_tsqr_factor(ws, iws, dt, dc, nc, w, ch, stream);
    if (e == hipSuccess) e = launch_thin_nn(ws, iws, dn + batch, dnc + n0, n1, THIN_CH, stream);
    if (e == hipSuccess) e = launch_thin_nn(ws, iws, dn + 2 * batch, dnc + n0 + n1, n2, THIN_CH, stream);
    if (e == hipSuccess) e = launch_tsqr_apply(ws, iws, dt, da, dc, nc, w, ch, w, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Q, ws + offQ, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(R, ws + offR, sizeof(double) * batch * ww, hipMemcpyDeviceToDevice, stream);
    std::vector<int> flags((size_t)batch * iper);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), iws, sizeof(int) * flags.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_cholqr: ") + hipGetErrorString(e));
    for (int b = 0; b < batch; ++b) fell_back[b] = flags[(size_t)b * iper + nodes];
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_debug_panel_qr(const double* P, int32_t batch, int64_t h, int32_t w, double* Q,
                                           double* R, int32_t* fell_back, hipStream_t stream) {
    using hsvd_detail::set_error;
    if (!P || !Q || !R || !fell_back || batch < 1 || h < 1 || w < 1 || w > kPanelQrMaxW ||
        w > kTsqrMaxW || h > (1 << 26))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_panel_qr: bad argument");
    Scratch sc;
    const int ch = tsqr_chunk_rows(w);
    const int nch = (int)((h + ch - 1) / ch);
    const int nodes = tsqr_nodes(nch, tsqr_fanin(w));
    const int64_t hw = h * w, ww = (int64_t)w * w, slot = tsqr_slot_size(w);
    // arena: P | I | Q | TSQR storage | R | panel QR scratch
    const int64_t offP = 0, offI = offP + batch * hw, offQ = offI + ww, offS = offQ + batch * hw,
                  offR = offS + (int64_t)batch * nodes * slot, offX = offR + batch * ww,
                  tot = offX + 2 * batch * ww;
    const int iper = nodes + 1;
    double* ws = sc.get<double>(tot);
    int* iws = sc.get<int>((size_t)batch * iper);
    TsqrTask* dt = sc.get<TsqrTask>(batch);
    ApplyTask* da = sc.get<ApplyTask>(batch);
    ChunkRef* dc = sc.get<ChunkRef>((size_t)batch * nch);
    if (!ws || !iws || !dt || !da || !dc) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    std::vector<TsqrTask> tt(batch);
    std::vector<ApplyTask> at(batch);
    std::vector<ChunkRef> cr;
    for (int b = 0; b < batch; ++b) {
        TsqrTask t{};
        t.p_off = offP + b * hw;
        t.store_off = offS + (int64_t)b * nodes * slot;
        t.r_out = offR + b * ww;
        t.h = (int)h;
        t.p_ld = (int)h;
        t.nch = nch;
        t.chunk0 = b * nch;
        t.cnt_off = b * iper;
        t.levels = tsqr_levels(nch, tsqr_fanin(w));
        t.cq_flag = b * iper + nodes;
        t.pq_q_off = offQ + b * hw;
        t.pq_q_ld = (int)h;
        t.pq_scr = offX + 2 * b * ww;
        tt[b] = t;
        ApplyTask a{};                                   // Householder fallback: Q = Q_H I
        a.tsqr = b;
        a.x_off = offI;
        a.out_off = offQ + b * hw;
        a.out_ld = (int)h;
        a.add_u_off = -1;
        at[b] = a;
        for (int c = 0; c < nch; ++c) cr.push_back({b, c});
    }
    std::vector<double> I((size_t)ww, 0.0);
    for (int i = 0; i < w; ++i) I[(size_t)i * w + i] = 1.0;
    hipError_t e = hipMemcpyAsync(ws + offP, P, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + offI, I.data(), sizeof(double) * ww, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(iws, 0, sizeof(int) * batch * iper, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tt.data(), sizeof(TsqrTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(da, at.data(), sizeof(ApplyTask) * batch, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, cr.data(), sizeof(ChunkRef) * cr.size(), hipMemcpyHostToDevice, stream);
    const int nc = (int)cr.size();
    if (e == hipSuccess) e = launch_panel_qr(ws, iws, dt, batch, w, 1, stream);
    if (e == hipSuccess) e = launch_tsqr_factor(ws, iws, dt, dc, nc, w, ch, stream);
    if (e == hipSuccess) e = launch_tsqr_apply(ws, iws, dt, da, dc, nc, w, ch, w, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Q, ws + offQ, sizeof(double) * batch * hw, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(R, ws + offR, sizeof(double) * batch * ww, hipMemcpyDeviceToDevice, stream);
    std::vector<int> flags((size_t)batch * iper);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), iws, sizeof(int) * flags.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_panel_qr: ") + hipGetErrorString(e));
    for (int b = 0; b < batch; ++b) fell_back[b] = flags[(size_t)b * iper + nodes];
    return HSVD_OK;
}

extern "C" hsvd_status hsvd_debug_probe(int32_t kind, void* buf, int64_t bytes, int32_t iters, double* ms_host,
                                        double* work_host, hipStream_t stream) {
    using hsvd_detail::set_error;
    const bool mem = kind == 0 || kind == 1;
    if (!ms_host || !work_host || kind < 0 || kind > 4 ||
        (mem && (!buf || bytes < 32 || ((uintptr_t)buf & 15))) || (!mem && (iters < 1 || iters > (1 << 24))))
        return set_error(HSVD_ERR_INVALID, "hsvd_debug_probe: bad argument");
    Scratch sc;
    float* sink = sc.get<float>(2048);
    if (!sink) return set_error(HSVD_ERR_ALLOC, "scratch allocation failed");
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    double work = 0.0;
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    if (e == hipSuccess) e = launch_probe(kind, buf, bytes, iters, sink, &work, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    for (hipEvent_t x : ev)
        if (x) hipEventDestroy(x);
    if (e != hipSuccess) return set_error(HSVD_ERR_HIP, std::string("hsvd_debug_probe: ") + hipGetErrorString(e));
    *ms_host = ms;
    *work_host = work;
    return HSVD_OK;
}
