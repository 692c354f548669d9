// C ABI and plan construction for the hierarchical MAT SVD (arXiv:1710.02812).
//
// A plan fixes everything that does not depend on the values of A: the balanced
// p x q partition (Algorithm 1 slicing, with the grid given as counts), the
// pairwise merge schedule of both trees (Algorithm 1, DoMergeOfSlices: neighbours
// (0,1), (2,3), ... left to right, an odd last node carried up), the layout of
// every panel in one device arena, and the task tables of each launch.  Ranks
// chosen by the truncation rule stay on the device; kernels read them, so an
// execute is a fixed sequence of launches with no host round trip (except when
// Algorithm 2 stops on a tolerance: one 4-byte read of the device's decision per
// iteration from the second on).
//
// Execute = the stages below, in order:
//   leaves      : Y = A_b Omega, then alternately QR and products with A_b^T / A_b
//                 (randomised range finder with power steps), QR of the last
//                 product, Jacobi core -> (U_b, s_b, r_b) per block;
//   column tree : per level, for all slabs at once: CGS2 projection coefficients
//                 C = U1^T U2, complement Q = U2 - U1 C (twice), TSQR of Q,
//                 Jacobi core of E = [[S1, C S2],[0, R S2]], U = U1 T + Q X;
//   re-project  : W_i^T = A_i^T U_i, TSQR, Jacobi -> (V_i, s_i) (Algorithm 1);
//   row tree    : the same merge on the V panels (height n);
//   projection  : Y = A V (split over column blocks), TSQR, Jacobi with rotations
//                 -> U = Q_Y Z, V = V J (Section 3, left vectors by projection);
//   refinement  : optional Algorithm 2 iterations (a fixed count, or until the
//                 singular values change by at most refine_eps between two);
//   output      : sign normalisation and the row-major U, S, Vt writes.
#include "../../include/hsvd.h"
#include "hsvd_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <mutex>
#include <string>
#include <random>
#include <vector>

using namespace hsvd;

namespace {

thread_local std::string g_last_error;

hsvd_status fail(hsvd_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
}  // namespace

namespace hsvd_detail {
hsvd_status set_error(hsvd_status st, const std::string& msg) { return fail(st, msg); }
}

namespace {

hsvd_status hip_fail(hipError_t e, const char* what) {
    return fail(HSVD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

enum StageKind { ST_GEMM, ST_TSQR_F, ST_TSQR_A, ST_GRAM, ST_REDUCE, ST_NN, ST_SUM, ST_CORE, ST_ENERGY, ST_CQ1, ST_CQ2,
                 ST_FEAT, ST_LEAFCHECK, ST_PQR, ST_GRAMX, ST_ESUM };

struct Stage {
    StageKind kind;
    int op = 0;          // gemm op
    int n = 0;           // tiles / chunks / tasks
    int w = 0, ch = 0, c = 0, N = 0;
    int maxdim = 0, with_v = 0;
    int bf16 = 0;        // gemm on the bfloat16 matrix cores
    int f32 = 0;         // gemm on the float32 matrix cores
    int64_t off = 0, off2 = 0;   // energy: output offset; features: sigma and energy offsets
    size_t tasks_off = 0, refs_off = 0, tsqr_off = 0;   // byte offsets in the task blob
    int guard = -1;      // int-arena slot: the stage is skipped while it holds non-zero
    int step = 0;        // leaf check: the power step it follows
    int need_r = 0;      // panel QR: R is formed
    int a64 = 0;         // passes over a float64 matrix held in the arena (the Gram matrix)
    // > 0: the stage belongs to leaf class `branch` of a plan whose leaves have several
    // sketch widths; the classes of a run of such stages are independent and run on
    // streams of their own between a fork and a join
    int branch = 0;
    int done_slot = -1;  // leaf check: int-arena slot of its leaf class's "all converged"
    int pw = 0;          // panel width of the matrices the stage works on
    int ordered = 0;     // panel QR: the tasks run in the dispatch order at order_off
    size_t order_off = 0;
    int64_t e_part = -1; // gemm (op 0, float64 matrix cores): per-tile partial block energies
    int tx = 2, ty = 2;  // thin gram / nn: 64-column tiles of the widest X and Y
};

int pow2floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

int tsqr_chunk(int w, int /*c*/) { return tsqr_chunk_rows(w); }


}  // namespace

// One matrix of a plan: shape, grid, rank cap and the balanced split points.
struct MatDesc {
    // The plan works on the logical matrix: the input itself, or its transpose when the
    // plan merges column slabs last (trans; Section 3: the order of the two sets of MAT
    // operations).  m, n, p, q, rs, cs are logical; the input is (trans ? n x m : m x n).
    int64_t m = 0, n = 0;
    int p = 0, q = 0, k = 0;
    int pw = 0;                    // width of the matrix's panels (its rank class's max k)
    bool trans = false;
    std::vector<int64_t> rs, cs;
    int64_t brow(int i) const { return rs[i + 1] - rs[i]; }
    int64_t bcol(int j) const { return cs[j + 1] - cs[j]; }
};

// Values chosen by the plan-time autotuner (0: the defaults).
struct Tuning { int thin_rows = 0, merge_qr = 0, leaf_qr = 0; float ms = 0.0f; };

struct hsvd_plan_st {
    std::vector<MatDesc> mats;     // one for hsvd_plan, count for hsvd_plan_batched
    int kind = 0;                  // 0: SVD plan, 1: block-feature plan
    bool trans = false;            // every matrix is handled transposed (column slabs merged last)
    // Gram plans (hsvd_plan_gram): the trees decompose G = X^T X (matrix 0, held in the
    // arena at gram_off, pointer-table entry 0 points there); the projection, Algorithm 2
    // and the output use X (matrix 1).  ntree: the matrices the trees run on.
    bool gram = false;
    int64_t gram_off = -1;
    int ntree = 0;
    std::vector<int> leaf_width;   // per-block sketch widths (width plans), else empty
    std::vector<int> leaf_rank_slots, leaf_flag_slots;   // per block of matrix 0
    int64_t energy_off = -1;       // block energies (width and feature plans)
    double tol = 0.0;
    hsvd_options opt{};
    int W = 0, L = 0, g = 0;       // panel width (max k), leaf sketch width, products per leaf
    // leaves' power steps until converged (power_steps = -1 on float64 plans): at most
    // leaf_cap steps; per class of leaves an int-arena slot turns 1 once every leaf of
    // the class has passed its test, and the class's later steps return at once (the
    // slot is cleared at each execute)
    int leaf_cap = 0;
    std::vector<int> reset_slots;  // int-arena slots cleared at the start of each execute
    size_t reset_off = 0;          // their device copy in the task blob

    // arenas (host-side bookkeeping)
    int64_t ws_elems = 0;
    int iws_elems = 0;
    std::vector<unsigned char> blob;
    std::vector<Stage> stages;
    std::vector<std::pair<int64_t, std::vector<double>>> ws_init;   // constant panels
    std::vector<std::pair<int64_t, double>> ws_fill;                  // (off, count) zero fills
    std::vector<std::pair<int64_t, int64_t>> zero_ranges;
    int64_t omega_off = 0, omega_count = 0;

    // device
    int device = 0;
    double* ws = nullptr;
    int* iws = nullptr;
    unsigned* flags = nullptr;
    void* dblob = nullptr;
    void** dptrs = nullptr;        // pointer table: A, U, S, Vt per matrix
    std::vector<void*> host_ptrs;  // its last uploaded contents
    hipStream_t last_stream = nullptr;
    bool executed = false;
    bool external = false;         // device state not allocated by the plan (not freed)
    bool ws_borrowed = false;      // arena and int arena in a caller buffer (hsvd_set_workspace)
    // learned block rank (hsvd_set_rank_model): network parameters (device), the
    // feature plan and its output, the predictions, the width plan of the last execute
    // and its widths, the plan whose result the last execute returned (this plan when
    // the plain widths stood in), and the refits that execute ran
    float* rm_params = nullptr;
    float* rm_feat = nullptr;
    float* rm_pred = nullptr;
    hsvd_plan_st* rm_features = nullptr;
    hsvd_plan_st* rm_wplan = nullptr;
    std::vector<int> rm_widths;
    hsvd_plan_st* rm_ran = nullptr;
    int rm_refits = 0, rm_plain = 0;
    // the launch sequence captured on the first execute (opt.graph), replayed after
    hipStream_t cap_stream = nullptr;
    int thin_ch = THIN_CH;                    // rows per chunk of the thin products
    int merge_qr = 0;                         // bit 0 / bit 1: panel QR in column / row merges
    int leaf_qr = 0;                          // leaves' QR: 0 by panel count, 1 panel QR, 2 TSQR
    bool merging_rows = false;                // build time: the row-merge tree is being built
    int tuned = 0;                            // 1: thin_ch and merge_qr came from the autotuner
    float tuned_ms = 0.0f;                    // its median execute time (ms)
    int nbranch = 0;                          // leaf classes run concurrently (0: none)
    std::vector<hipStream_t> bstreams;        // one per class
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    // final
    std::vector<OutputArgs> outs;  // per matrix
    std::vector<int> rank_slots;   // per matrix
    size_t outs_off = 0;           // OutputArgs array in the task blob
    int kmax = 0, mmax = 0, nmax = 0;

    // Algorithm 2 stopped on a tolerance (refine_eps > 0, >= 2 iterations): the stages
    // of iteration t end at seg_end[t]; after iteration t >= 1 a check compares its
    // singular values with those of t - 1 (check_off[t]: RefineCheck array in the
    // blob), and the output of an execute stopped after iteration t reads
    // step_outs_off[t] with ranks in step_rank_slots[t].  Empty otherwise.
    std::vector<size_t> seg_end, check_off, step_outs_off;
    std::vector<std::vector<int>> step_rank_slots;
    int check_slot = -1;
    int refine_done = 0;           // iterations of Algorithm 2 run by the last execute

    // optional per-launch timing: events[i] .. events[i+1] bracket launch i
    bool profiling = false;
    std::vector<hipEvent_t> events;
    std::vector<int> event_kind;

    int64_t alloc(int64_t elems) {
        const int64_t off = ws_elems;
        ws_elems += (elems + 31) / 32 * 32;
        return off;
    }
    int ialloc(int count) {
        const int off = iws_elems;
        iws_elems += count;
        return off;
    }
    template <typename T>
    size_t put(const std::vector<T>& v) {
        size_t off = (blob.size() + 255) / 256 * 256;
        blob.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

namespace {

// ------------------------------------------------------------------ schedule builders
struct Node {            // a factor node: panel (h x W, ld), sigma (W), rank slot
    int64_t panel, sig;
    int ld, h, rank;
    int mat;             // matrix of the batch
};

struct TsqrBuild {
    std::vector<TsqrTask> tasks;
    std::vector<ChunkRef> chunks;
    bool cholqr = false;     // some task takes the Cholesky QR fast path
    bool pqr = false;        // some task takes the one-launch panel QR
};

// The leaves' QR: the one-launch panel QR (one work-group per panel) pays when the
// panels of a launch fill at least half the chip; fewer panels keep the chunked
// Householder TSQR, whose chunks spread each panel over several work-groups
// (hsvd_options.leaf_qr overrides the choice).
bool use_panel_qr(const hsvd_plan_st& P, size_t npanels, int64_t hmax, int w) {
    (void)hmax;
    if (w > kPanelQrMaxW || P.leaf_qr == 2) return false;
    return P.leaf_qr == 1 || npanels >= 128;
}

// Tall panels wider than the Cholesky QR's 64 columns (slab re-projections, projections
// and Algorithm 2 panels of rank caps above 64): the one-launch panel QR, one work-group
// per panel, when a launch has at least 128 of them; fewer keep the chunked Householder
// TSQR, whose chunks spread each panel over several work-groups.
bool wide_panel_qr(size_t npanels, int w) {
    return w > 64 && w <= kPanelQrMaxW && npanels >= 128;
}

// Adds TSQR bookkeeping for a panel; returns index into tb.tasks.  cholqr: the panel
// (expected well-conditioned) first tries two Cholesky QR passes, the Householder
// kernels running only if they fall back (panels up to 64 columns).
int add_tsqr(hsvd_plan_st& P, TsqrBuild& tb, int64_t panel, int h, int ld, int w, int ch,
             bool cholqr = false, int64_t pq_dest = -1, int pq_ld = 0) {
    TsqrTask t{};
    t.p_off = panel;
    t.h = h;
    t.p_ld = ld;
    t.nch = (h + ch - 1) / ch;
    t.chunk0 = (int)tb.chunks.size();
    const int nodes = tsqr_nodes(t.nch, tsqr_fanin(w));
    t.levels = tsqr_levels(t.nch, tsqr_fanin(w));
    t.store_off = P.alloc((int64_t)nodes * tsqr_slot_size(w));
    t.cnt_off = P.ialloc(nodes);
    t.r_out = P.alloc((int64_t)w * w);
    if (cholqr && w <= 64 && ch == tsqr_chunk_rows(w)) {
        t.cq_off = P.alloc(cq_size(w, t.nch, h));
        t.cq_flag = P.ialloc(1);
        t.cq_cnt = P.ialloc(std::max(1, cq_nodes(t.nch)));
        tb.cholqr = true;
    } else if (pq_dest >= 0 && w <= kPanelQrMaxW) {
        // one-launch panel QR: Q to pq_dest, R to r_out; Householder on its fallback
        t.pq_q_off = pq_dest;
        t.pq_q_ld = pq_ld;
        t.pq_scr = P.alloc(2 * (int64_t)w * w);
        t.cq_flag = P.ialloc(1);
        tb.pqr = true;
    }
    for (int c = 0; c < t.nch; ++c) tb.chunks.push_back({(int)tb.tasks.size(), c});
    tb.tasks.push_back(t);
    return (int)tb.tasks.size() - 1;
}

void push_thin(hsvd_plan_st& P, StageKind kind, std::vector<ThinTask> tasks);

// span_only (panel QR): the factor only has to span the panel for the next power step,
// so the panel QR stops after its shifted first pass.
void push_tsqr_factor(hsvd_plan_st& P, const TsqrBuild& tb, int w, int ch, bool need_r = true,
                      bool span_only = false) {
    if (tb.pqr) {
        Stage q{};
        q.kind = ST_PQR;
        q.n = (int)tb.tasks.size();
        q.w = w;
        q.ch = ch;
        q.need_r = span_only && !need_r ? kPqrSpanOnly : need_r ? 1 : 0;
        q.tasks_off = P.put(tb.tasks);
        // one work-group per panel: the tallest panels first, so that a launch over
        // panels of uneven heights (a batch) does not end on its longest work-groups
        std::vector<int> order(tb.tasks.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return tb.tasks[a].h > tb.tasks[b].h; });
        q.ordered = 1;
        q.order_off = P.put(order);
        P.stages.push_back(q);
    }
    if (tb.cholqr) {
        // pass 1 (G = P^T P, R1, M1 = R1^-1), Q1 = P M1, pass 2 (Q1^T Q1, R = R2 R1, M2)
        Stage c{};
        c.kind = ST_CQ1;
        c.n = (int)tb.chunks.size();
        c.w = w;
        c.ch = ch;
        c.tasks_off = P.put(tb.tasks);
        c.refs_off = P.put(tb.chunks);
        P.stages.push_back(c);
        std::vector<ThinTask> q1;
        for (const TsqrTask& t : tb.tasks) {
            if (t.cq_flag < 0) continue;
            ThinTask x{};
            x.x_off = t.p_off; x.x_ld = t.p_ld;
            x.c_off = t.cq_off + (int64_t)w * w; x.c_ld = w;                    // M1
            x.y_off = t.cq_off + cq_q1(w, t.nch); x.y_ld = t.h;                 // Q1
            x.h = t.h; x.wx = w; x.wy = w; x.accumulate = 0; x.cond = t.cq_flag;
            q1.push_back(x);
        }
        if (!q1.empty()) push_thin(P, ST_NN, q1);
        c.kind = ST_CQ2;
        P.stages.push_back(c);
    }
    Stage s{};
    s.kind = ST_TSQR_F;
    s.n = (int)tb.chunks.size();
    s.w = w;
    s.ch = ch;
    s.tasks_off = P.put(tb.tasks);
    s.refs_off = P.put(tb.chunks);
    P.stages.push_back(s);
}

// Apply stage for tasks applying the factors of `tb` (one ApplyTask per tsqr task, in order).
void push_tsqr_apply(hsvd_plan_st& P, const TsqrBuild& tb, const std::vector<ApplyTask>& at,
                     int w, int ch, int c) {
    if (tb.pqr) {
        // out = Q X (+ U1 T) from the explicit Q; an apply of the identity into the panel
        // the panel QR already wrote is nothing more to do
        std::vector<ThinTask> nn;
        for (const ApplyTask& a : at) {
            const TsqrTask& t = tb.tasks[a.tsqr];
            if (t.pq_q_off < 0 || (a.out_off == t.pq_q_off && a.add_u_off < 0)) continue;
            ThinTask y{};
            y.x_off = t.pq_q_off; y.x_ld = t.pq_q_ld;
            y.c_off = a.x_off; y.c_ld = w;
            y.y_off = a.out_off; y.y_ld = a.out_ld;
            y.h = t.h; y.wx = w; y.wy = c; y.accumulate = 0; y.cond = t.cq_flag;
            if (a.add_u_off >= 0) {
                y.x2_off = a.add_u_off; y.x2_ld = a.add_u_ld;
                y.c2_off = a.add_t_off; y.c2_ld = a.add_w;
                y.wx2 = a.add_w;
            }
            nn.push_back(y);
        }
        if (!nn.empty()) push_thin(P, ST_NN, nn);
    }
    if (tb.cholqr) {
        // out = Q X + U1 T with Q = Q1 M2: C = M2 X (w x c), then out = Q1 C + U1 T
        std::vector<ThinTask> n1, n2;
        for (const ApplyTask& a : at) {
            const TsqrTask& t = tb.tasks[a.tsqr];
            if (t.cq_flag < 0) continue;
            const int64_t C = P.alloc((int64_t)w * c);
            ThinTask x{};
            x.x_off = t.cq_off + 2 * (int64_t)w * w; x.x_ld = w;                  // M2
            x.c_off = a.x_off; x.c_ld = w;
            x.y_off = C; x.y_ld = w;
            x.h = w; x.wx = w; x.wy = c; x.accumulate = 0; x.cond = t.cq_flag;
            n1.push_back(x);
            ThinTask y{};
            y.x_off = t.cq_off + cq_q1(w, t.nch); y.x_ld = t.h;                   // Q1
            y.c_off = C; y.c_ld = w;
            y.y_off = a.out_off; y.y_ld = a.out_ld;
            y.h = t.h; y.wx = w; y.wy = c; y.accumulate = 0; y.cond = t.cq_flag;
            if (a.add_u_off >= 0) {
                y.x2_off = a.add_u_off; y.x2_ld = a.add_u_ld;
                y.c2_off = a.add_t_off; y.c2_ld = a.add_w;
                y.wx2 = a.add_w;
            }
            n2.push_back(y);
        }
        if (!n1.empty()) push_thin(P, ST_NN, n1);
        if (!n2.empty()) push_thin(P, ST_NN, n2);
    }
    Stage s{};
    s.kind = ST_TSQR_A;
    s.n = (int)tb.chunks.size();
    s.w = w;
    s.ch = ch;
    s.c = c;
    s.tsqr_off = P.put(tb.tasks);
    s.tasks_off = P.put(at);
    s.refs_off = P.put(tb.chunks);   // chunk.task indexes both arrays
    P.stages.push_back(s);
}

// A pass over A on the float64 matrix cores (mma 0, 64 x 64 tiles), the bfloat16 ones
// (mma 1) or the float32 ones (mma 2; both in strips of 256 rows holding every column).
enum { MMA_F64 = 0, MMA_BF16 = 1, MMA_F32 = 2 };
// Returns each task's range of tiles (first, count) in the launch.
std::vector<std::pair<int, int>> push_gemm(hsvd_plan_st& P, int op, std::vector<GemmTask> tasks, int N,
                                           int mma = MMA_F64) {
    if (P.trans) op = 1 - op;                     // logical A_blk X = (stored block)^T X
    std::vector<TileRef> tiles;
    std::vector<std::pair<int, int>> ranges;
    const bool strip = mma != MMA_F64;
    const int nct = strip ? 1 : gemm_f64_col_tiles(N);
    const int th = strip ? kBf16TileRows : 64;
    for (size_t t = 0; t < tasks.size(); ++t) {
        const int out_rows = (op == 0) ? tasks[t].rows : tasks[t].cols;
        const int nrt = (out_rows + th - 1) / th;
        tasks[t].tiles = nrt;
        ranges.push_back({(int)tiles.size(), nrt * nct});
        for (int i = 0; i < nrt * nct; ++i) tiles.push_back({(int)t, i});
    }
    Stage s{};
    s.kind = ST_GEMM;
    s.bf16 = mma == MMA_BF16 ? 1 : 0;
    s.f32 = mma == MMA_F32 ? 1 : 0;
    s.a64 = (P.gram && !tasks.empty() && tasks[0].mat == 0) ? 1 : 0;
    s.op = op;
    s.n = (int)tiles.size();
    s.N = N;
    s.tasks_off = P.put(tasks);
    s.refs_off = P.put(tiles);
    P.stages.push_back(s);
    return ranges;
}

// A sketch pass Y = A_blk X on the float64 matrix cores (the stage just pushed) that
// also yields each block's energy ||A_blk||_F^2: its tiles write partial sums, and a
// small stage adds each task's partials in tile order into outs[task].
bool energy_fusable(const hsvd_plan_st& P) { return !P.trans && P.opt.precision != HSVD_MIXED_BF16; }
void fuse_energy(hsvd_plan_st& P, const std::vector<std::pair<int, int>>& ranges,
                 const std::vector<int64_t>& outs) {
    const int ntiles = P.stages.back().n;
    const int64_t part = P.alloc(std::max(ntiles, 1));
    P.stages.back().e_part = part;
    std::vector<EnergySum> es;
    for (size_t u = 0; u < ranges.size(); ++u) es.push_back({outs[u], ranges[u].first, ranges[u].second});
    Stage s{};
    s.kind = ST_ESUM;
    s.n = (int)es.size();
    s.off2 = part;
    s.w = ntiles;
    s.tasks_off = P.put(es);
    P.stages.push_back(s);
}

// Thin ops over row chunks: builds chunk refs for each task.
void push_thin(hsvd_plan_st& P, StageKind kind, std::vector<ThinTask> tasks) {
    std::vector<ChunkRef> chunks;
    for (size_t t = 0; t < tasks.size(); ++t) {
        tasks[t].nch = (tasks[t].h + P.thin_ch - 1) / P.thin_ch;
        tasks[t].chunk0 = (int)chunks.size();
        if (kind != ST_REDUCE)
            for (int c = 0; c < tasks[t].nch; ++c) chunks.push_back({(int)t, c});
    }
    Stage s{};
    s.kind = kind;
    s.n = (kind == ST_REDUCE) ? (int)tasks.size() : (int)chunks.size();
    if (kind == ST_REDUCE)
        for (const ThinTask& t : tasks) s.w = std::max(s.w, t.wx * t.wy);
    s.tx = s.ty = 1;                              // no work-groups for tiles no task has
    for (const ThinTask& t : tasks) {
        if (t.wx > 64) s.tx = 2;
        if (t.wy > 64) s.ty = 2;
    }
    s.tasks_off = P.put(tasks);
    s.refs_off = P.put(chunks);
    P.stages.push_back(s);
}

// One work-group per core: the widest cores first (a merge core's width is at most twice
// its rank cap), so that a launch over cores of uneven widths does not end on its longest
// work-groups; cores of one width keep their order.
void push_core(hsvd_plan_st& P, std::vector<CoreTask> tasks, int maxdim, int with_v) {
    auto width = [](const CoreTask& t) { return t.mode == CORE_MERGE ? 2 * t.kcap : t.dim; };
    std::stable_sort(tasks.begin(), tasks.end(),
                     [&](const CoreTask& a, const CoreTask& b) { return width(a) > width(b); });
    Stage s{};
    s.kind = ST_CORE;
    s.n = (int)tasks.size();
    s.maxdim = maxdim;
    s.with_v = with_v;
    s.tasks_off = P.put(tasks);
    P.stages.push_back(s);
}

// The tree cores' orthogonality threshold: loose on mixed-precision and float32-storage
// plans, below their inputs' own rounding.
double tree_orth_tol(const hsvd_plan_st& P) {
    return P.opt.precision == HSVD_MIXED_BF16 ? kMixedOrthTol : P.opt.precision == HSVD_FP32 ? kF32OrthTol : 0.0;
}

CoreTask core_defaults(const hsvd_plan_st& P, int k) {
    CoreTask c{};
    c.rank_in = -1;
    c.u_off = c.t_off = c.v_off = -1;
    c.rank1 = c.rank2 = -1;
    c.kcap = k;
    c.rule = P.opt.rule;
    c.tol = P.tol;
    c.floor_cols = -1;
    c.fixed_rank_slot = -1;
    c.energy_off = -1;
    c.flag_slot = -1;
    return c;
}

// Identity (w x w) constant panel.
int64_t identity_panel(hsvd_plan_st& P, int w) {
    const int64_t off = P.alloc((int64_t)w * w);
    std::vector<double> I((size_t)w * w, 0.0);
    for (int i = 0; i < w; ++i) I[(size_t)i * w + i] = 1.0;
    P.ws_init.push_back({off, I});
    return off;
}

// A pass task over the logical block at logical offset a_off (r0 * n + c0), rows x cols.
// For a transposed plan the block is stored transposed in the input (rows and cols
// swap, the leading dimension is the logical m) and push_gemm flips the product.
GemmTask gemm_task(const hsvd_plan_st& P, int mat, int64_t a_off, int64_t rows, int64_t cols) {
    const MatDesc& M = P.mats[mat];
    GemmTask t{};
    t.mat = mat;
    if (!M.trans) {
        t.lda = M.n;
        t.a_off = a_off;
        t.rows = (int)rows;
        t.cols = (int)cols;
    } else {
        const int64_t r0 = a_off / M.n, c0 = a_off % M.n;
        t.lda = M.m;
        t.a_off = c0 * M.m + r0;
        t.rows = (int)cols;
        t.cols = (int)rows;
    }
    return t;
}

// One level of merges (all pairs of all trees at this level), in place of the
// right operand's panel for the complement.
std::vector<Node> merge_level(hsvd_plan_st& P, const std::vector<std::pair<Node, Node>>& pairs) {
    const int W = P.W;
    const int chq = tsqr_chunk(W, W);
    std::vector<Node> outs;
    std::vector<ThinTask> gram1, red1, sub1, gram2, red2, sub2;
    TsqrBuild tb;
    std::vector<CoreTask> cores, wide;
    std::vector<ApplyTask> applies;
    for (const auto& pr : pairs) {
        const Node& a = pr.first;
        const Node& b = pr.second;
        const int h = a.h;
        const int nch = (h + P.thin_ch - 1) / P.thin_ch;
        const int64_t part = P.alloc((int64_t)nch * W * W);
        const int64_t C1 = P.alloc((int64_t)W * W), C2 = P.alloc((int64_t)W * W);
        const int64_t Cacc = P.alloc((int64_t)W * W);
        ThinTask g{};
        g.x_off = a.panel; g.x_ld = a.ld;
        g.y_off = b.panel; g.y_ld = b.ld;
        g.h = h; g.wx = W; g.wy = W;
        g.part_off = part; g.acc_off = -1;
        gram1.push_back(g);
        ThinTask r = g;
        r.c_off = C1; r.c_ld = W; r.acc_off = Cacc; r.accumulate = 0;
        red1.push_back(r);
        ThinTask sb{};
        sb.x_off = a.panel; sb.x_ld = a.ld;
        sb.y_off = b.panel; sb.y_ld = b.ld;
        sb.c_off = C1; sb.c_ld = W;
        sb.h = h; sb.wx = W; sb.wy = W; sb.accumulate = 2; sb.acc_off = -1;
        sub1.push_back(sb);
        gram2.push_back(g);
        ThinTask r2 = r;
        r2.c_off = C2; r2.accumulate = 1;
        red2.push_back(r2);
        ThinTask sb2 = sb;
        sb2.c_off = C2;
        sub2.push_back(sb2);

        // the complement's QR: Cholesky QR, or the one-launch panel QR (explicit Q)
        const bool pq = ((P.merge_qr >> (P.merging_rows ? 1 : 0)) & 1) && W <= kPanelQrMaxW;
        const int ti = add_tsqr(P, tb, b.panel, h, b.ld, W, chq, !pq, pq ? P.alloc((int64_t)h * W) : -1, h);
        Node o{};
        o.mat = a.mat;
        o.h = h;
        o.ld = a.ld;
        o.panel = P.alloc((int64_t)o.ld * W);
        o.sig = P.alloc(W);
        o.rank = P.ialloc(1);
        const int64_t T = P.alloc((int64_t)W * W), X = P.alloc((int64_t)W * W);
        CoreTask c = core_defaults(P, P.mats[a.mat].k);
        c.mode = CORE_MERGE;
        c.s1_off = a.sig; c.s2_off = b.sig;
        c.c_off = Cacc; c.c_ld = W;
        c.r_off = tb.tasks[ti].r_out; c.r_ld = W;
        c.rank1 = a.rank; c.rank2 = b.rank;
        c.t_off = T; c.t_ld = W;
        c.u_off = X; c.u_ld = W;
        c.sig_off = o.sig;
        c.out_w = W;
        c.rank_out = o.rank;
        c.floor_rows = h;
        c.floor_cols = -1;
        c.precond = 1;
        c.orth_tol = tree_orth_tol(P);
        // a core of two children of rank above kCoreMaxN / 2 may exceed the LDS-resident
        // cores: such merges go to the wide cores, with a scratch panel each
        if (2 * P.mats[a.mat].k > kCoreMaxN) {
            c.scr_off = P.alloc(kWideScratch);
            wide.push_back(c);
        } else {
            cores.push_back(c);
        }
        ApplyTask ap{};
        ap.tsqr = ti;
        ap.x_off = X;
        ap.out_off = o.panel;
        ap.out_ld = o.ld;
        ap.add_u_off = a.panel;
        ap.add_u_ld = a.ld;
        ap.add_t_off = T;
        ap.add_w = W;
        applies.push_back(ap);
        outs.push_back(o);
    }
    push_thin(P, ST_GRAM, gram1);
    push_thin(P, ST_REDUCE, red1);
    push_thin(P, ST_NN, sub1);
    push_thin(P, ST_GRAM, gram2);
    push_thin(P, ST_REDUCE, red2);
    push_thin(P, ST_NN, sub2);
    push_tsqr_factor(P, tb, W, chq);
    if (!cores.empty()) push_core(P, cores, std::min(2 * W, kCoreMaxN), 0);
    if (!wide.empty()) push_core(P, wide, 2 * W, 0);
    push_tsqr_apply(P, tb, applies, W, chq, W);
    return outs;
}

// Runs the merge tree of several independent forests level by level.
std::vector<Node> merge_forest(hsvd_plan_st& P, std::vector<std::vector<Node>> trees) {
    for (;;) {
        bool any = false;
        std::vector<std::pair<Node, Node>> pairs;
        std::vector<std::vector<int>> where(trees.size());
        for (size_t t = 0; t < trees.size(); ++t) {
            const auto& lv = trees[t];
            if (lv.size() > 1) any = true;
            for (size_t i = 0; i + 1 < lv.size(); i += 2) {
                where[t].push_back((int)pairs.size());
                pairs.push_back({lv[i], lv[i + 1]});
            }
        }
        if (!any) break;
        const std::vector<Node> outs = merge_level(P, pairs);
        for (size_t t = 0; t < trees.size(); ++t) {
            const auto& lv = trees[t];
            if (lv.size() <= 1) continue;
            std::vector<Node> nxt;
            for (int idx : where[t]) nxt.push_back(outs[idx]);
            if (lv.size() % 2) nxt.push_back(lv.back());
            trees[t] = nxt;
        }
    }
    std::vector<Node> roots;
    for (auto& t : trees) roots.push_back(t[0]);
    return roots;
}

// Leaf pipeline for one class of leaves sharing the sketch width w: randomised range
// finder with power steps (Y = A_b Omega_w, then alternately QR and products with
// A_b^T / A_b), QR of the last product, Jacobi core -> (U_b, s_b, r_b).
struct Leaf { int mat, i, j, w; int64_t rowsz, colsz, aoff; };
struct LeafPanels { int64_t Y, Z, Qy, Qz; };

// Leaf core task of leaf b (sketch width w): Jacobi on R^T of the last QR of Y = A_b Q_z,
// writing the node's sigma and rank and the w x W rotation U_R (at ur).
CoreTask leaf_core_task(hsvd_plan_st& P, const Leaf& l, int b, int w, int64_t r_out, int mode,
                        int64_t ur, Node& nd) {
    const int W = P.W;
    nd.mat = l.mat;
    nd.h = (int)l.rowsz;
    nd.ld = (int)l.rowsz;
    nd.panel = P.alloc(l.rowsz * W);
    nd.sig = P.alloc(W);
    nd.rank = P.ialloc(1);
    CoreTask c = core_defaults(P, P.mats[l.mat].k);
    c.mode = mode;
    c.dim = w;
    c.m_off = r_out;
    c.m_ld = w;
    c.u_off = ur;
    c.u_ld = w;
    c.sig_off = nd.sig;
    c.out_w = W;
    c.rank_out = nd.rank;
    c.floor_rows = (int)l.rowsz;
    c.floor_cols = (int)l.colsz;
    c.precond = 1;                // left vectors only: LQ of R first (fewer sweeps)
    c.orth_tol = tree_orth_tol(P);
    if (P.energy_off >= 0 && l.mat == 0) {
        c.energy_off = P.energy_off + b;
        c.flag_slot = P.ialloc(1);
        P.leaf_flag_slots[b] = c.flag_slot;
    }
    if (l.mat == 0) P.leaf_rank_slots[b] = nd.rank;
    return c;
}

// Leaves whose power steps run until their subspaces have converged.  After the
// sketch Y = A_b Omega and its QR, step t = 1, 2, ... forms Q_y, Z = A_b^T Q_y, its QR
// and Q_z, Y = A_b Q_z and its QR, and the leaf core on R; a device-side test then
// bounds how far one more step could still turn each leaf's kept subspace (subspace
// iteration shrinks the angle to the block's top-r subspace by (s_{w+1} / s_r)^2 per
// step, estimated from the core's values).  Every step reuses the same panels, so
// whichever step passed the test last, the final apply U_b = Q_y U_R reads its
// factors; the launches of the steps after it return at once.
void leaf_converge(hsvd_plan_st& P, const std::vector<Leaf>& leaves, const std::vector<int>& ids, int w,
                   int ch, int64_t I_w, const std::vector<LeafPanels>& pan, std::vector<Node>& nodes) {
    const int W = P.W;
    TsqrBuild tby, tbz;
    int64_t hmax = 1;
    for (int b : ids) hmax = std::max({hmax, leaves[b].rowsz, leaves[b].colsz});
    const bool pq = use_panel_qr(P, ids.size(), hmax, w);
    for (size_t u = 0; u < ids.size(); ++u) {
        const Leaf& l = leaves[ids[u]];
        add_tsqr(P, tby, pan[u].Y, (int)l.rowsz, (int)l.rowsz, w, ch, false, pq ? pan[u].Qy : -1, (int)l.rowsz);
        add_tsqr(P, tbz, pan[u].Z, (int)l.colsz, (int)l.colsz, w, ch, false, pq ? pan[u].Qz : -1, (int)l.colsz);
    }
    push_tsqr_factor(P, tby, w, ch);
    std::vector<CoreTask> cores;
    std::vector<LeafCheck> checks;
    std::vector<ApplyTask> aqy, aqz, aout;
    std::vector<GemmTask> gz, gy;
    for (size_t u = 0; u < ids.size(); ++u) {
        const int b = ids[u];
        const Leaf& l = leaves[b];
        const int64_t ur = P.alloc((int64_t)w * W);
        CoreTask c = leaf_core_task(P, l, b, w, tby.tasks[u].r_out, CORE_UPPER, ur, nodes[b]);
        c.sigall_off = P.alloc(w);
        cores.push_back(c);
        LeafCheck k{};
        k.sig_off = c.sigall_off;
        k.w = w;
        k.kcap = P.mats[l.mat].k;
        k.rule = P.opt.rule;
        k.tol = P.tol;
        k.floor_rows = (int)l.rowsz;
        k.floor_cols = (int)l.colsz;
        checks.push_back(k);
        ApplyTask a{};
        a.tsqr = (int)u;
        a.x_off = I_w;
        a.add_u_off = -1;
        a.out_off = pan[u].Qy; a.out_ld = (int)l.rowsz;
        aqy.push_back(a);
        a.out_off = pan[u].Qz; a.out_ld = (int)l.colsz;
        aqz.push_back(a);
        a.x_off = ur;
        a.out_off = nodes[b].panel; a.out_ld = nodes[b].ld;
        aout.push_back(a);
        GemmTask x = gemm_task(P, l.mat, l.aoff, l.rowsz, l.colsz);
        x.x_off = pan[u].Qy; x.x_ld = (int)l.rowsz;          // Z = A_b^T Q_y
        x.y_off = pan[u].Z; x.y_ld = (int)l.colsz;
        gz.push_back(x);
        x.x_off = pan[u].Qz; x.x_ld = (int)l.colsz;          // Y = A_b Q_z
        x.y_off = pan[u].Y; x.y_ld = (int)l.rowsz;
        gy.push_back(x);
    }
    const size_t checks_off = P.put(checks);
    // this class's "every leaf has converged" slot (cleared at the start of an execute)
    const int done = P.ialloc(1);
    P.reset_slots.push_back(done);
    for (int t = 1; t <= P.leaf_cap; ++t) {
        const size_t first = P.stages.size();
        push_tsqr_apply(P, tby, aqy, w, ch, w);
        push_gemm(P, 1, gz, w);
        push_tsqr_factor(P, tbz, w, ch, false);
        push_tsqr_apply(P, tbz, aqz, w, ch, w);
        push_gemm(P, 0, gy, w);
        push_tsqr_factor(P, tby, w, ch);
        push_core(P, cores, w, 0);
        Stage s{};
        s.kind = ST_LEAFCHECK;
        s.n = (int)checks.size();
        s.tasks_off = checks_off;
        s.step = t;
        s.done_slot = done;
        P.stages.push_back(s);
        if (t > 1)
            for (size_t i = first; i < P.stages.size(); ++i) P.stages[i].guard = done;
    }
    push_tsqr_apply(P, tby, aout, w, ch, W);
}

void leaf_pipeline(hsvd_plan_st& P, const std::vector<Leaf>& leaves, const std::vector<int>& ids, int w,
                   int64_t omega_ld, std::vector<Node>& nodes) {
    const int W = P.W, g = P.g;
    const bool bf16 = P.opt.precision == HSVD_MIXED_BF16;
    const int64_t I_w = identity_panel(P, w);
    std::vector<LeafPanels> pan(ids.size());
    for (size_t u = 0; u < ids.size(); ++u) {
        const Leaf& l = leaves[ids[u]];
        pan[u] = {P.alloc(l.rowsz * w), P.alloc(l.colsz * w), P.alloc(l.rowsz * w), P.alloc(l.colsz * w)};
    }
    {
        std::vector<GemmTask> gt;
        for (size_t u = 0; u < ids.size(); ++u) {
            const Leaf& l = leaves[ids[u]];
            GemmTask t = gemm_task(P, l.mat, l.aoff, l.rowsz, l.colsz);
            t.x_off = P.omega_off; t.x_ld = (int)omega_ld;
            t.y_off = pan[u].Y; t.y_ld = (int)l.rowsz;
            gt.push_back(t);
        }
        const auto ranges = push_gemm(P, 0, gt, w, bf16 ? MMA_BF16 : MMA_F64);
        if (P.energy_off >= 0 && energy_fusable(P)) {   // width plans: the leaves' energies
            std::vector<int64_t> outs;
            for (int b : ids) outs.push_back(P.energy_off + b);
            fuse_energy(P, ranges, outs);
        }
    }
    const int ch = tsqr_chunk(w, std::max(w, W));
    if (P.leaf_cap > 0) {
        leaf_converge(P, leaves, ids, w, ch, I_w, pan, nodes);
        return;
    }
    TsqrBuild tb_last;
    int64_t hmax = 1;
    for (int b : ids) hmax = std::max({hmax, leaves[b].rowsz, leaves[b].colsz});
    const bool pq = use_panel_qr(P, ids.size(), hmax, w);
    for (int t = 1; t <= g; ++t) {
        const bool prev_is_y = ((t - 1) % 2 == 0);
        TsqrBuild tb;
        for (size_t u = 0; u < ids.size(); ++u) {
            const Leaf& l = leaves[ids[u]];
            if (prev_is_y)
                add_tsqr(P, tb, pan[u].Y, (int)l.rowsz, (int)l.rowsz, w, ch, false, pq ? pan[u].Qy : -1,
                         (int)l.rowsz);
            else
                add_tsqr(P, tb, pan[u].Z, (int)l.colsz, (int)l.colsz, w, ch, false, pq ? pan[u].Qz : -1,
                         (int)l.colsz);
        }
        // the sketch's own QR (float32 storage and mixed plans, one power step): its Q
        // only sets the subspace that Z = A_b^T Q spans, so the panel QR stops after its
        // shifted pass (a well-conditioned basis of the same span); the later QRs stay full
        push_tsqr_factor(P, tb, w, ch, t == g, t == 1 && t < g && P.opt.precision != HSVD_FP64);
        if (t == g) { tb_last = tb; break; }
        std::vector<ApplyTask> at;
        for (size_t u = 0; u < ids.size(); ++u) {
            const Leaf& l = leaves[ids[u]];
            ApplyTask a{};
            a.tsqr = (int)u;
            a.x_off = I_w;
            a.out_off = prev_is_y ? pan[u].Qy : pan[u].Qz;
            a.out_ld = prev_is_y ? (int)l.rowsz : (int)l.colsz;
            a.add_u_off = -1;
            at.push_back(a);
        }
        push_tsqr_apply(P, tb, at, w, ch, w);
        std::vector<GemmTask> gt;
        for (size_t u = 0; u < ids.size(); ++u) {
            const Leaf& l = leaves[ids[u]];
            GemmTask x = gemm_task(P, l.mat, l.aoff, l.rowsz, l.colsz);
            if (prev_is_y) {            // Z = A_b^T Qy
                x.x_off = pan[u].Qy; x.x_ld = (int)l.rowsz;
                x.y_off = pan[u].Z; x.y_ld = (int)l.colsz;
            } else {                    // Y = A_b Qz
                x.x_off = pan[u].Qz; x.x_ld = (int)l.colsz;
                x.y_off = pan[u].Y; x.y_ld = (int)l.rowsz;
            }
            gt.push_back(x);
        }
        push_gemm(P, prev_is_y ? 1 : 0, gt, w, bf16 ? MMA_BF16 : MMA_F64);
    }
    const bool last_is_y = ((g - 1) % 2 == 0);
    std::vector<CoreTask> cores;
    std::vector<int64_t> ur(ids.size());
    for (size_t u = 0; u < ids.size(); ++u) {
        const int b = ids[u];
        ur[u] = P.alloc((int64_t)w * W);
        cores.push_back(leaf_core_task(P, leaves[b], b, w, tb_last.tasks[u].r_out,
                                       last_is_y ? CORE_UPPER : CORE_UPPER_T, ur[u], nodes[b]));
    }
    push_core(P, cores, w, 0);
    if (last_is_y) {
        std::vector<ApplyTask> at;
        for (size_t u = 0; u < ids.size(); ++u) {
            ApplyTask a{};
            a.tsqr = (int)u;
            a.x_off = ur[u];
            a.out_off = nodes[ids[u]].panel;
            a.out_ld = nodes[ids[u]].ld;
            a.add_u_off = -1;
            at.push_back(a);
        }
        push_tsqr_apply(P, tb_last, at, w, ch, W);
    } else {
        std::vector<ThinTask> nn;
        for (size_t u = 0; u < ids.size(); ++u) {
            const Leaf& l = leaves[ids[u]];
            ThinTask t{};
            t.x_off = pan[u].Qy; t.x_ld = (int)l.rowsz;
            t.c_off = ur[u]; t.c_ld = w;
            t.y_off = nodes[ids[u]].panel; t.y_ld = nodes[ids[u]].ld;
            t.h = (int)l.rowsz; t.wx = w; t.wy = W;
            t.accumulate = 0; t.acc_off = -1;
            nn.push_back(t);
        }
        push_thin(P, ST_NN, nn);
    }
}

// Sketch width of a matrix of a batched plan: its own k + oversample (within its
// smallest block side and the leaf kernels' limit), rounded up to a multiple of 8 so
// that the batch has few width classes (each class is one pipeline of launches, the
// classes run concurrently).
int batch_width(const hsvd_plan_st& P, const MatDesc& M) {
    int64_t bmin = INT64_MAX;
    for (int i = 0; i < M.p; ++i) bmin = std::min(bmin, M.brow(i));
    for (int j = 0; j < M.q; ++j) bmin = std::min(bmin, M.bcol(j));
    const int lim = (int)std::min<int64_t>(bmin, kTsqrMaxW);
    const int w = ((M.k + P.opt.oversample + 7) / 8) * 8;
    return std::max(1, std::min(w, lim));
}

// Leaves of every block of every matrix (of the matrices in `only`, when given).
// Sketch width P.L for all, or the per-block widths of a width plan, or a batched
// plan's per-matrix widths (leaves grouped by width: one pipeline per class, run as
// concurrent branches when branch_classes).  Width plans first compute every block's
// energy for the leaf check.  One Gaussian test matrix serves every leaf of the plan.
// Returns one forest per (matrix, row slab), matrices in order, slabs top to bottom.
std::vector<std::vector<Node>> build_leaves(hsvd_plan_st& P, const std::vector<int>* only = nullptr,
                                            bool branch_classes = true) {
    auto leaf_w = [&](const MatDesc& M, int i, int j) {
        return !P.leaf_width.empty() ? P.leaf_width[(size_t)i * M.q + j]
               : P.ntree > 1 ? batch_width(P, M) : P.L;
    };
    int64_t bcmax = 1;
    int wmax = 1;
    for (int mi = 0; mi < P.ntree; ++mi) {
        const MatDesc& M = P.mats[mi];
        for (int i = 0; i < M.p; ++i)
            for (int j = 0; j < M.q; ++j) {
                bcmax = std::max(bcmax, M.bcol(j));
                wmax = std::max(wmax, leaf_w(M, i, j));
            }
    }
    if (P.omega_count == 0) {
        P.omega_count = bcmax * wmax;
        P.omega_off = P.alloc(P.omega_count);
    }
    std::vector<Leaf> leaves;
    for (int mi = 0; mi < P.ntree; ++mi) {
        if (only && std::find(only->begin(), only->end(), mi) == only->end()) continue;
        const MatDesc& M = P.mats[mi];
        for (int i = 0; i < M.p; ++i)
            for (int j = 0; j < M.q; ++j) {
                Leaf l{};
                l.mat = mi;
                l.i = i; l.j = j;
                l.rowsz = M.brow(i);
                l.colsz = M.bcol(j);
                l.aoff = M.rs[i] * M.n + M.cs[j];
                l.w = leaf_w(M, i, j);
                leaves.push_back(l);
            }
    }
    if (P.leaf_rank_slots.empty()) {
        P.leaf_rank_slots.assign((size_t)P.mats[0].p * P.mats[0].q, -1);
        P.leaf_flag_slots.assign((size_t)P.mats[0].p * P.mats[0].q, -1);
    }
    if (!P.leaf_width.empty()) {
        P.energy_off = P.alloc((int64_t)leaves.size());
    }
    if (!P.leaf_width.empty() && !energy_fusable(P)) {   // else summed in the sketch pass
        std::vector<GemmTask> et;
        for (const Leaf& l : leaves) et.push_back(gemm_task(P, l.mat, l.aoff, l.rowsz, l.colsz));
        Stage s{};
        s.kind = ST_ENERGY;
        s.n = (int)et.size();
        s.off = P.energy_off;
        s.tasks_off = P.put(et);
        P.stages.push_back(s);
    }
    std::vector<int> widths;
    for (const Leaf& l : leaves)
        if (std::find(widths.begin(), widths.end(), l.w) == widths.end()) widths.push_back(l.w);
    std::sort(widths.begin(), widths.end());
    std::vector<Node> nodes(leaves.size());
    for (size_t c = 0; c < widths.size(); ++c) {
        std::vector<int> ids;
        for (size_t b = 0; b < leaves.size(); ++b)
            if (leaves[b].w == widths[c]) ids.push_back((int)b);
        const size_t first = P.stages.size();
        leaf_pipeline(P, leaves, ids, widths[c], bcmax, nodes);
        if (widths.size() > 1 && branch_classes)
            for (size_t i = first; i < P.stages.size(); ++i) P.stages[i].branch = (int)c + 1;
    }
    if (widths.size() > 1 && branch_classes) P.nbranch = (int)widths.size();
    std::vector<std::vector<Node>> slabs;
    int prev_mat = -1, prev_i = -1;
    for (size_t b = 0; b < leaves.size(); ++b) {
        if (leaves[b].mat != prev_mat || leaves[b].i != prev_i) {
            slabs.emplace_back();
            prev_mat = leaves[b].mat;
            prev_i = leaves[b].i;
        }
        slabs.back().push_back(nodes[b]);
    }
    return slabs;
}

// Slab re-projection: V_i, s_i = SVD(U_i^T A_i), for the column-tree root of every
// (matrix, slab) in the order build_leaves produced them.  Returns one row forest
// per matrix present, in matrix order.
std::vector<std::vector<Node>> build_reprojection(hsvd_plan_st& P, const std::vector<Node>& roots) {
    const int W = P.W;
    const int ch = tsqr_chunk(W, W);
    std::vector<GemmTask> gt;
    TsqrBuild tb;
    std::vector<int64_t> Zs(roots.size());
    std::vector<int> slab(roots.size());
    for (size_t i = 0; i < roots.size(); ++i) {
        const int mi = roots[i].mat;
        slab[i] = (i > 0 && roots[i - 1].mat == mi) ? slab[i - 1] + 1 : 0;
        const MatDesc& M = P.mats[mi];
        const int n = (int)M.n;
        Zs[i] = P.alloc((int64_t)n * W);
        GemmTask t = gemm_task(P, mi, M.rs[slab[i]] * M.n, M.brow(slab[i]), n);
        t.x_off = roots[i].panel; t.x_ld = roots[i].ld;
        t.y_off = Zs[i]; t.y_ld = n;
        gt.push_back(t);
    }
    push_gemm(P, 1, gt, W, P.opt.precision == HSVD_MIXED_BF16 ? MMA_BF16 : MMA_F64);
    const bool pq = wide_panel_qr(roots.size(), W);
    for (size_t i = 0; i < roots.size(); ++i) {
        const int n = (int)P.mats[roots[i].mat].n;
        add_tsqr(P, tb, Zs[i], n, n, W, ch, true, pq ? P.alloc((int64_t)n * W) : -1, n);
    }
    push_tsqr_factor(P, tb, W, ch);
    std::vector<CoreTask> cores;
    std::vector<ApplyTask> at;
    std::vector<std::vector<Node>> out(P.ntree);
    for (size_t i = 0; i < roots.size(); ++i) {
        const int mi = roots[i].mat;
        const int n = (int)P.mats[mi].n;
        Node nd{};
        nd.mat = mi;
        nd.h = n;
        nd.ld = n;
        nd.panel = P.alloc((int64_t)n * W);
        nd.sig = P.alloc(W);
        nd.rank = P.ialloc(1);
        const int64_t X = P.alloc((int64_t)W * W);
        CoreTask c = core_defaults(P, P.mats[mi].k);
        c.mode = CORE_UPPER;
        c.dim = W;
        c.m_off = tb.tasks[i].r_out;
        c.m_ld = W;
        c.rank_in = roots[i].rank;
        c.orth_tol = tree_orth_tol(P);
        c.u_off = X;
        c.u_ld = W;
        c.sig_off = nd.sig;
        c.out_w = W;
        c.rank_out = nd.rank;
        c.floor_rows = n;
        c.floor_cols = 0;
        cores.push_back(c);
        ApplyTask a{};
        a.tsqr = (int)i;
        a.x_off = X;
        a.out_off = nd.panel;
        a.out_ld = n;
        a.add_u_off = -1;
        at.push_back(a);
        out[mi].push_back(nd);
    }
    push_core(P, cores, W, 0);
    push_tsqr_apply(P, tb, at, W, ch, W);
    // the forests of the matrices present (a rank class of a batched plan holds some)
    std::vector<std::vector<Node>> present;
    for (auto& f : out)
        if (!f.empty()) present.push_back(std::move(f));
    return present;
}

struct Factors { int64_t U, V, sig; int rank; int mat; };

// Left vectors by projection, for every matrix: Y = A V (split over column
// blocks), TSQR(Y) = Q R, Jacobi on R (with rotations J): U = Q Z, V <- V J.
std::vector<Factors> build_projection(hsvd_plan_st& P, const std::vector<Node>& vs) {
    const int W = P.W;
    const int ch = tsqr_chunk(W, W);
    std::vector<GemmTask> gt;
    std::vector<ThinTask> sums;
    std::vector<int64_t> Ys(vs.size());
    for (size_t mi = 0; mi < vs.size(); ++mi) {
        const MatDesc& M = P.mats[vs[mi].mat];
        const int64_t m = M.m, n = M.n;
        const int64_t parts = P.alloc((int64_t)M.q * m * W);
        for (int i = 0; i < M.p; ++i)
            for (int j = 0; j < M.q; ++j) {
                GemmTask t = gemm_task(P, vs[mi].mat, M.rs[i] * n + M.cs[j], M.brow(i), M.bcol(j));
                t.x_off = vs[mi].panel + M.cs[j];
                t.x_ld = vs[mi].ld;
                t.y_off = parts + (int64_t)j * m * W + M.rs[i];
                t.y_ld = (int)m;
                gt.push_back(t);
            }
        Ys[mi] = P.alloc(m * W);
        ThinTask s{};
        s.x_off = parts; s.x_ld = (int)m;
        s.c_ld = (int)(m * W);      // stride between partials
        s.wx = M.q; s.wy = W;
        s.y_off = Ys[mi]; s.y_ld = (int)m;
        s.h = (int)m;
        s.acc_off = -1;
        sums.push_back(s);
    }
    // mixed plans: float32-accurate products on the float32 matrix cores
    push_gemm(P, 0, gt, W, P.opt.precision == HSVD_MIXED_BF16 ? MMA_F32 : MMA_F64);
    push_thin(P, ST_SUM, sums);
    TsqrBuild tb;
    const bool pq = wide_panel_qr(vs.size(), W);
    for (size_t mi = 0; mi < vs.size(); ++mi) {
        const int m = (int)P.mats[vs[mi].mat].m;
        add_tsqr(P, tb, Ys[mi], m, m, W, ch, true, pq ? P.alloc((int64_t)m * W) : -1, m);
    }
    push_tsqr_factor(P, tb, W, ch);
    std::vector<Factors> fs(vs.size());
    std::vector<CoreTask> cores;
    std::vector<ApplyTask> at;
    std::vector<ThinTask> nns;
    for (size_t mi = 0; mi < vs.size(); ++mi) {
        const MatDesc& M = P.mats[vs[mi].mat];
        const int64_t m = M.m, n = M.n;
        Factors& f = fs[mi];
        f.mat = vs[mi].mat;
        f.U = P.alloc(m * W);
        f.V = P.alloc(n * W);
        f.sig = P.alloc(W);
        f.rank = P.ialloc(1);
        const int64_t X = P.alloc((int64_t)W * W), J = P.alloc((int64_t)W * W);
        CoreTask c = core_defaults(P, M.k);
        c.mode = CORE_UPPER;
        c.dim = W;
        c.m_off = tb.tasks[mi].r_out;
        c.m_ld = W;
        c.rank_in = vs[mi].rank;
        c.u_off = X; c.u_ld = W;
        c.v_off = J; c.v_ld = W;
        c.sig_off = f.sig;
        c.out_w = W;
        c.rank_out = f.rank;
        c.floor_rows = (int)m;
        c.floor_cols = -1;
        c.fixed_rank_slot = vs[mi].rank;
        cores.push_back(c);
        ApplyTask a{};
        a.tsqr = (int)mi;
        a.x_off = X;
        a.out_off = f.U;
        a.out_ld = (int)m;
        a.add_u_off = -1;
        at.push_back(a);
        ThinTask nn{};
        nn.x_off = vs[mi].panel; nn.x_ld = vs[mi].ld;
        nn.c_off = J; nn.c_ld = W;
        nn.y_off = f.V; nn.y_ld = (int)n;
        nn.h = (int)n; nn.wx = W; nn.wy = W;
        nn.accumulate = 0; nn.acc_off = -1;
        nns.push_back(nn);
    }
    push_core(P, cores, W, 1);
    push_tsqr_apply(P, tb, at, W, ch, W);
    push_thin(P, ST_NN, nns);
    return fs;
}

// One Algorithm 2 step per matrix from (U_i = left vectors of A V):
// W^T = A^T U_i = Q R; Jacobi on R with rotations J: V~ = Q Z, U^ = U_i J, S~.
std::vector<Factors> build_refine_step(hsvd_plan_st& P, const std::vector<Factors>& in) {
    const int W = P.W;
    const int ch = tsqr_chunk(W, W);
    std::vector<GemmTask> gt;
    std::vector<ThinTask> sums;
    std::vector<int64_t> Zs(in.size());
    for (size_t mi = 0; mi < in.size(); ++mi) {
        const MatDesc& M = P.mats[in[mi].mat];
        const int64_t m = M.m, n = M.n;
        const int64_t parts = P.alloc((int64_t)M.p * n * W);
        for (int i = 0; i < M.p; ++i) {
            GemmTask t = gemm_task(P, in[mi].mat, M.rs[i] * n, M.brow(i), n);
            t.x_off = in[mi].U + M.rs[i];
            t.x_ld = (int)m;
            t.y_off = parts + (int64_t)i * n * W;
            t.y_ld = (int)n;
            gt.push_back(t);
        }
        Zs[mi] = P.alloc(n * W);
        ThinTask s{};
        s.x_off = parts; s.x_ld = (int)n;
        s.c_ld = (int)(n * W);
        s.wx = M.p; s.wy = W;
        s.y_off = Zs[mi]; s.y_ld = (int)n;
        s.h = (int)n;
        s.acc_off = -1;
        sums.push_back(s);
    }
    push_gemm(P, 1, gt, W, P.opt.precision == HSVD_MIXED_BF16 ? MMA_F32 : MMA_F64);
    push_thin(P, ST_SUM, sums);
    TsqrBuild tb;
    const bool pq = wide_panel_qr(in.size(), W);
    for (size_t mi = 0; mi < in.size(); ++mi) {
        const int n = (int)P.mats[in[mi].mat].n;
        add_tsqr(P, tb, Zs[mi], n, n, W, ch, true, pq ? P.alloc((int64_t)n * W) : -1, n);
    }
    push_tsqr_factor(P, tb, W, ch);
    std::vector<Factors> fs(in.size());
    std::vector<CoreTask> cores;
    std::vector<ApplyTask> at;
    std::vector<ThinTask> nns;
    for (size_t mi = 0; mi < in.size(); ++mi) {
        const MatDesc& M = P.mats[in[mi].mat];
        const int64_t m = M.m, n = M.n;
        Factors& f = fs[mi];
        f.mat = in[mi].mat;
        f.U = P.alloc(m * W);
        f.V = P.alloc(n * W);
        f.sig = P.alloc(W);
        f.rank = P.ialloc(1);
        const int64_t X = P.alloc((int64_t)W * W), J = P.alloc((int64_t)W * W);
        CoreTask c = core_defaults(P, M.k);
        c.mode = CORE_UPPER;
        c.dim = W;
        c.m_off = tb.tasks[mi].r_out;
        c.m_ld = W;
        c.rank_in = in[mi].rank;
        c.u_off = X; c.u_ld = W;
        c.v_off = J; c.v_ld = W;
        c.sig_off = f.sig;
        c.out_w = W;
        c.rank_out = f.rank;
        c.floor_rows = (int)n;
        c.floor_cols = -1;
        c.fixed_rank_slot = in[mi].rank;
        cores.push_back(c);
        ApplyTask a{};
        a.tsqr = (int)mi;
        a.x_off = X;
        a.out_off = f.V;
        a.out_ld = (int)n;
        a.add_u_off = -1;
        at.push_back(a);
        ThinTask nn{};
        nn.x_off = in[mi].U; nn.x_ld = (int)m;
        nn.c_off = J; nn.c_ld = W;
        nn.y_off = f.U; nn.y_ld = (int)m;
        nn.h = (int)m; nn.wx = W; nn.wy = W;
        nn.accumulate = 0; nn.acc_off = -1;
        nns.push_back(nn);
    }
    push_core(P, cores, W, 1);
    push_tsqr_apply(P, tb, at, W, ch, W);
    push_thin(P, ST_NN, nns);
    return fs;
}

// G = X^T X into the arena: partial Grams over row chunks of X (upper-triangle tiles,
// mirrored), summed by the thin-sum kernel unless there is a single chunk.  For the sum
// the n^2 contiguous elements are viewed as wy <= 128 columns of H rows (the last one
// running past n^2 into slack that is allocated and whose sums are not used).
void build_gram(hsvd_plan_st& P) {
    const MatDesc& X = P.mats[1];
    const int64_t m = X.m, n = X.n, nn = n * n;
    const int T = (int)((n + 63) / 64), ntile = T * (T + 1) / 2;
    int64_t nch = std::max<int64_t>(1, std::min<int64_t>((1024 + ntile - 1) / ntile, (m + 255) / 256));
    const int64_t rows = (m + nch - 1) / nch;
    nch = (m + rows - 1) / rows;
    const int64_t H = (nn + 127) / 128, wy = (nn + H - 1) / H;
    P.gram_off = P.alloc(nch == 1 ? nn : wy * H);
    const int64_t parts = nch == 1 ? P.gram_off : P.alloc(nch * nn + wy * H);
    std::vector<GramRef> refs;
    for (int64_t c = 0; c < nch; ++c)
        for (int a = 0; a < T; ++a)
            for (int b = a; b < T; ++b) refs.push_back({a, b, (int)c, 0});
    Stage s{};
    s.kind = ST_GRAMX;
    s.n = (int)refs.size();
    s.off = parts;
    s.off2 = rows;
    s.tasks_off = P.put(refs);
    P.stages.push_back(s);
    if (nch > 1) {                                // only for n < 2880 (fewer than 1024 tiles)
        ThinTask t{};
        t.x_off = parts; t.x_ld = (int)H;
        t.c_ld = (int)nn;
        t.wx = (int)nch; t.wy = (int)wy;
        t.y_off = P.gram_off; t.y_ld = (int)H;
        t.h = (int)H;
        t.acc_off = -1;
        push_thin(P, ST_SUM, {t});
    }
}

// Output table of factors ff, one entry per matrix (sign slots of its own).
std::vector<OutputArgs> output_table(hsvd_plan_st& P, const std::vector<Factors>& ff, std::vector<int>& ranks) {
    std::vector<OutputArgs> outs;
    ranks.clear();
    for (size_t mi = 0; mi < ff.size(); ++mi) {
        const MatDesc& M = P.mats[ff[mi].mat];
        OutputArgs o{};
        // a transposed plan's right vectors are the input's left vectors
        o.u_off = M.trans ? ff[mi].V : ff[mi].U;
        o.v_off = M.trans ? ff[mi].U : ff[mi].V;
        o.sig_off = ff[mi].sig;
        o.u_ld = (int)(M.trans ? M.n : M.m);
        o.v_ld = (int)(M.trans ? M.m : M.n);
        o.m = (int)(M.trans ? M.n : M.m);
        o.n = (int)(M.trans ? M.m : M.n);
        o.k = M.k;
        o.rank_slot = ff[mi].rank;
        o.sign_off = P.ialloc(M.k);
        outs.push_back(o);
        ranks.push_back(ff[mi].rank);
    }
    return outs;
}

void output_extents(hsvd_plan_st& P, const std::vector<Factors>& f) {
    P.kmax = P.mmax = P.nmax = 0;
    for (size_t mi = 0; mi < f.size(); ++mi) {
        const MatDesc& M = P.mats[f[mi].mat];
        P.kmax = std::max(P.kmax, M.k);
        P.mmax = std::max<int>(P.mmax, (int)std::max(M.m, M.n));
        P.nmax = std::max<int>(P.nmax, (int)std::max(M.m, M.n));
    }
}

// Next projection input from an Algorithm 2 step's factors (V and sigma).
std::vector<Node> nodes_of(const hsvd_plan_st& P, const std::vector<Factors>& f) {
    std::vector<Node> vs(f.size());
    for (size_t mi = 0; mi < f.size(); ++mi) {
        vs[mi].mat = f[mi].mat;
        vs[mi].panel = f[mi].V;
        vs[mi].ld = (int)P.mats[f[mi].mat].n;
        vs[mi].h = (int)P.mats[f[mi].mat].n;
        vs[mi].rank = f[mi].rank;
        vs[mi].sig = f[mi].sig;
    }
    return vs;
}

// Rank classes of a batched plan: the matrices grouped by leaf sketch width (adjacent
// widths merged into at most kRankClasses groups).  Each class gets the panel width of
// its largest rank cap, so that matrices of small rank do not pay for the batch's
// largest, and its stages form a branch of their own (the classes are independent).
// One class for everything else, and for plans stopping Algorithm 2 on refine_eps
// (whose host checks split the stage list into segments).
constexpr int kRankClasses = 4;
std::vector<std::vector<int>> rank_classes(const hsvd_plan_st& P, bool eps_stop) {
    std::vector<std::vector<int>> cls;
    if (P.ntree < 2 || P.gram || !P.leaf_width.empty() || eps_stop) {
        cls.emplace_back();
        for (int mi = 0; mi < P.ntree; ++mi) cls[0].push_back(mi);
        return cls;
    }
    std::vector<int> widths;
    for (int mi = 0; mi < P.ntree; ++mi) {
        const int w = batch_width(P, P.mats[mi]);
        if (std::find(widths.begin(), widths.end(), w) == widths.end()) widths.push_back(w);
    }
    std::sort(widths.begin(), widths.end());
    const int nw = (int)widths.size(), nc = std::min(nw, kRankClasses);
    cls.resize(nc);
    for (int mi = 0; mi < P.ntree; ++mi) {
        const int wi = (int)(std::find(widths.begin(), widths.end(), batch_width(P, P.mats[mi])) - widths.begin());
        cls[(size_t)wi * nc / nw].push_back(mi);
    }
    return cls;
}

hsvd_status build_plan(hsvd_plan_st& P) {
    if (P.gram) build_gram(P);
    const int steps = P.opt.refine_steps + (P.opt.precision == HSVD_MIXED_BF16 ? 1 : 0);
    const bool eps_stop = P.opt.refine_eps > 0.0 && steps >= 2;
    P.seg_end.clear();
    P.check_off.clear();
    P.step_outs_off.clear();
    P.step_rank_slots.clear();
    P.refine_done = steps;
    const std::vector<std::vector<int>> classes = rank_classes(P, eps_stop);
    if (classes.size() > 1) {
        // every class's whole pipeline with its own panel width, as a branch
        const int wall = P.W;
        std::vector<Factors> fall(P.ntree);
        for (size_t c = 0; c < classes.size(); ++c) {
            const std::vector<int>& ids = classes[c];
            int w = 1;
            for (int mi : ids) w = std::max(w, P.mats[mi].k);
            P.W = w;
            const size_t first = P.stages.size();
            auto slabs = build_leaves(P, &ids, false);
            P.merging_rows = false;
            auto col_roots = merge_forest(P, slabs);
            auto row_forests = build_reprojection(P, col_roots);
            P.merging_rows = true;
            auto row_roots = merge_forest(P, row_forests);
            std::vector<Factors> f = build_projection(P, row_roots);
            for (int it = 0; it < steps; ++it) {
                f = build_refine_step(P, f);
                if (it + 1 < steps) f = build_projection(P, nodes_of(P, f));
            }
            for (const Factors& x : f) fall[(size_t)x.mat] = x;
            for (int mi : ids) P.mats[mi].pw = w;
            for (size_t i = first; i < P.stages.size(); ++i) {
                P.stages[i].branch = (int)c + 1;
                P.stages[i].pw = w;
            }
        }
        P.W = wall;
        P.nbranch = (int)classes.size();
        output_extents(P, fall);
        P.outs = output_table(P, fall, P.rank_slots);
        P.outs_off = P.put(P.outs);
        return HSVD_OK;
    }
    auto slabs = build_leaves(P);
    P.merging_rows = false;
    auto col_roots = merge_forest(P, slabs);
    auto row_forests = build_reprojection(P, col_roots);
    P.merging_rows = true;
    auto row_roots = merge_forest(P, row_forests);
    if (P.gram)                                   // V-hat of G = X^T X is X's: project against X
        for (Node& r : row_roots) r.mat = 1;
    std::vector<Factors> f = build_projection(P, row_roots);
    if (eps_stop) P.check_slot = P.ialloc(1);
    // the first iteration is tested against Algorithm 1's singular values (the row
    // tree's root), each later one against the iteration before it
    std::vector<Factors> prev(f.size());
    // (a Gram plan's tree holds X^T X's values, X's squared: its first iteration is
    // tested against the projection's values, X's own)
    for (size_t mi = 0; mi < f.size(); ++mi) prev[mi].sig = P.gram ? f[mi].sig : row_roots[mi].sig;
    std::vector<OutputArgs> last_outs;
    for (int it = 0; it < steps; ++it) {
        f = build_refine_step(P, f);
        if (eps_stop) {
            P.seg_end.push_back(P.stages.size());
            std::vector<RefineCheck> checks;
            for (size_t mi = 0; mi < f.size(); ++mi) {
                RefineCheck c{};
                c.sig_old = prev[mi].sig;
                c.sig_new = f[mi].sig;
                c.rank_slot = f[mi].rank;
                checks.push_back(c);
            }
            P.check_off.push_back(P.put(checks));
            std::vector<int> ranks;
            last_outs = output_table(P, f, ranks);
            P.step_outs_off.push_back(P.put(last_outs));
            P.step_rank_slots.push_back(ranks);
            prev = f;
        }
        if (it + 1 < steps) f = build_projection(P, nodes_of(P, f));
    }
    for (Stage& st : P.stages) st.pw = P.W;
    for (MatDesc& M : P.mats) M.pw = P.W;
    output_extents(P, f);
    if (eps_stop) {
        // the last iteration's table doubles as the plan's output
        P.outs = last_outs;
        P.outs_off = P.step_outs_off.back();
        P.rank_slots = P.step_rank_slots.back();
    } else {
        P.outs = output_table(P, f, P.rank_slots);
        P.outs_off = P.put(P.outs);
    }
    return HSVD_OK;
}

// Block features (learned rank): energy of every block, a 16-column Gaussian sketch
// Y = A_b Omega_16, its TSQR and the singular values of R, then the 16 features.
void build_features(hsvd_plan_st& P) {
    const MatDesc& M = P.mats[0];
    const int nb = M.p * M.q;
    int64_t bcmax = 1;
    for (int j = 0; j < M.q; ++j) bcmax = std::max(bcmax, M.bcol(j));
    P.omega_count = bcmax * 16;
    P.omega_off = P.alloc(P.omega_count);
    P.energy_off = P.alloc(nb);
    const int64_t sigs = P.alloc(16LL * nb);
    std::vector<GemmTask> et, gt;
    std::vector<int64_t> Ys(nb), outs(nb);
    for (int i = 0; i < M.p; ++i)
        for (int j = 0; j < M.q; ++j) {
            const int b = i * M.q + j;
            GemmTask t = gemm_task(P, 0, M.rs[i] * M.n + M.cs[j], M.brow(i), M.bcol(j));
            et.push_back(t);
            Ys[b] = P.alloc(M.brow(i) * 16);
            outs[b] = P.energy_off + b;
            t.x_off = P.omega_off; t.x_ld = (int)bcmax;
            t.y_off = Ys[b]; t.y_ld = (int)M.brow(i);
            gt.push_back(t);
        }
    if (!energy_fusable(P)) {
        Stage se{};
        se.kind = ST_ENERGY;
        se.n = nb;
        se.off = P.energy_off;
        se.tasks_off = P.put(et);
        P.stages.push_back(se);
    }
    const auto ranges = push_gemm(P, 0, gt, 16);
    if (energy_fusable(P)) fuse_energy(P, ranges, outs);   // the energies in the sketch pass
    const int ch = tsqr_chunk(16, 16);
    TsqrBuild tb;
    for (int b = 0; b < nb; ++b) {
        const int h = (int)M.brow(b / M.q);
        add_tsqr(P, tb, Ys[b], h, h, 16, ch);
    }
    push_tsqr_factor(P, tb, 16, ch);
    std::vector<CoreTask> cores;
    for (int b = 0; b < nb; ++b) {
        CoreTask c = core_defaults(P, 16);
        c.rule = 0;
        c.tol = 0.0;
        c.mode = CORE_UPPER;
        c.dim = 16;
        c.m_off = tb.tasks[b].r_out;
        c.m_ld = 16;
        c.sig_off = sigs + 16LL * b;
        c.out_w = 16;
        c.rank_out = P.ialloc(1);
        c.floor_rows = (int)M.brow(b / M.q);
        c.floor_cols = 16;
        cores.push_back(c);
    }
    push_core(P, cores, 16, 0);
    Stage sf{};
    sf.kind = ST_FEAT;
    sf.n = nb;
    sf.off = sigs;
    sf.off2 = P.energy_off;
    P.stages.push_back(sf);
    P.kmax = P.mmax = P.nmax = 0;
    P.outs_off = P.put(P.outs);
}

// Host-side bounds check of every task in every stage against the arenas and A:
// each kernel's index range is recomputed here from the task fields, so a plan
// whose footprint leaves its buffers is rejected before anything is launched.
std::string validate_plan(const hsvd_plan_st& P) {
    const int64_t WS = P.ws_elems, IW = P.iws_elems;
    const unsigned char* b = P.blob.data();
    char msg[256];
    auto span = [&](const char* what, int64_t off, int64_t last, int64_t lim) -> bool {
        if (off < 0 || last >= lim) {
            snprintf(msg, sizeof msg, "%s out of bounds: off=%lld last=%lld limit=%lld", what,
                     (long long)off, (long long)last, (long long)lim);
            return false;
        }
        return true;
    };
    auto panel = [&](const char* what, int64_t off, int64_t ld, int64_t rows, int64_t cols) {
        if (rows <= 0 || cols <= 0) return true;
        if (ld < rows) { snprintf(msg, sizeof msg, "%s: ld %lld < rows %lld", what, (long long)ld, (long long)rows); return false; }
        return span(what, off, off + (cols - 1) * ld + rows - 1, WS);
    };
    for (size_t si = 0; si < P.stages.size(); ++si) {
        const Stage& s = P.stages[si];
        std::string err;
        switch (s.kind) {
            case ST_GEMM: {
                const GemmTask* T = (const GemmTask*)(b + s.tasks_off);
                const TileRef* R = (const TileRef*)(b + s.refs_off);
                int ntask = 0;
                for (int i = 0; i < s.n; ++i) ntask = std::max(ntask, R[i].task + 1);
                for (int i = 0; i < ntask; ++i) {
                    const GemmTask& t = T[i];
                    if (t.mat < 0 || t.mat >= (int)P.mats.size()) return "gemm matrix index";
                    const MatDesc& M = P.mats[t.mat];
                    const int64_t ld = M.trans ? M.m : M.n;     // the input's row length
                    if (t.lda != ld) return "gemm leading dimension";
                    if (!span("gemm A", t.a_off, t.a_off + (int64_t)(t.rows - 1) * ld + t.cols - 1, M.m * M.n)) return msg;
                    if (t.cols > ld || t.a_off % ld + t.cols > ld) return "gemm A block crosses a row";
                    const int xr = s.op == 0 ? t.cols : t.rows, yr = s.op == 0 ? t.rows : t.cols;
                    if (!panel("gemm X", t.x_off, t.x_ld, xr, s.N)) return msg;
                    if (!panel("gemm Y", t.y_off, t.y_ld, yr, s.N)) return msg;
                    const int th = (s.bf16 || s.f32) ? kBf16TileRows : 64;
                    if (t.tiles != (yr + th - 1) / th) return "gemm tile count";
                }
                const int nct = (s.bf16 || s.f32) ? 1 : gemm_f64_col_tiles(s.N);
                for (int i = 0; i < s.n; ++i)
                    if (R[i].tile < 0 || R[i].tile >= T[R[i].task].tiles * nct) return "gemm tile ref";
                if (s.e_part >= 0 && (s.op != 0 || s.bf16 || s.f32 || !span("gemm energy parts", s.e_part, s.e_part + s.n - 1, WS)))
                    return s.e_part >= 0 && (s.op != 0 || s.bf16 || s.f32) ? "fused energy on a pass other than A X" : msg;
                if (s.bf16 && P.opt.precision == HSVD_FP64) return "bf16 pass on a float64 plan";
                if (s.bf16 && s.N > kBf16MaxN) return "bf16 pass wider than its tile";
                if (s.f32 && (s.N > kBf16MaxN || P.opt.precision == HSVD_FP64)) return "float32 pass";
                break;
            }
            case ST_CQ1:
            case ST_TSQR_F:
            case ST_CQ2:
            case ST_TSQR_A: {
                const TsqrTask* T = (const TsqrTask*)(b + (s.kind != ST_TSQR_A ? s.tasks_off : s.tsqr_off));
                const ChunkRef* R = (const ChunkRef*)(b + s.refs_off);
                int ntask = 0;
                for (int i = 0; i < s.n; ++i) ntask = std::max(ntask, R[i].task + 1);
                if (s.w > kTsqrMaxW || s.c > kTsqrMaxW || s.ch < s.w || s.ch != tsqr_chunk_rows(s.w)) return "tsqr geometry";
                for (int i = 0; i < ntask; ++i) {
                    const TsqrTask& t = T[i];
                    const int nodes = tsqr_nodes(t.nch, tsqr_fanin(s.w));
                    if (t.levels != tsqr_levels(t.nch, tsqr_fanin(s.w))) return "tsqr levels";
                    if (t.nch != (t.h + s.ch - 1) / s.ch) return "tsqr chunk count";
                    if (!panel("tsqr panel", t.p_off, t.p_ld, t.h, s.w)) return msg;
                    if (!span("tsqr store", t.store_off, t.store_off + (int64_t)nodes * tsqr_slot_size(s.w) - 1, WS)) return msg;
                    if (!span("tsqr R", t.r_out, t.r_out + (int64_t)s.w * s.w - 1, WS)) return msg;
                    if (!span("tsqr counters", t.cnt_off, t.cnt_off + nodes - 1, IW)) return msg;
                    if (t.pq_q_off >= 0) {
                        if (s.kind == ST_CQ1 || s.kind == ST_CQ2) return "panel qr task in a Cholesky QR pass";
                        if (t.cq_flag < 0 || t.cq_flag >= IW) return "panel qr flag slot";
                    } else if (t.cq_flag >= 0) {
                        if (s.w > 64 || s.ch > 256) return "cholqr geometry";
                        if (!span("cholqr scratch", t.cq_off, t.cq_off + cq_size(s.w, t.nch, t.h) - 1, WS)) return msg;
                        if (t.cq_flag >= IW || t.cq_cnt < 0 || t.cq_cnt + std::max(1, cq_nodes(t.nch)) > IW)
                            return "cholqr slots";
                    } else if (s.kind == ST_CQ1 || s.kind == ST_CQ2) {
                        continue;                                   // no fast path: the passes skip it
                    }
                    if (s.kind == ST_TSQR_A) {
                        const ApplyTask& a = ((const ApplyTask*)(b + s.tasks_off))[i];
                        if (a.tsqr != i) return "apply/tsqr order";
                        if (!span("apply X", a.x_off, a.x_off + (int64_t)s.w * s.c - 1, WS)) return msg;
                        if (!panel("apply out", a.out_off, a.out_ld, t.h, s.c)) return msg;
                        if (a.add_u_off >= 0) {
                            if (!panel("apply U1", a.add_u_off, a.add_u_ld, t.h, a.add_w)) return msg;
                            if (!span("apply T", a.add_t_off, a.add_t_off + (int64_t)a.add_w * s.c - 1, WS)) return msg;
                        }
                    }
                }
                for (int i = 0; i < s.n; ++i)
                    if (R[i].chunk < 0 || R[i].chunk >= T[R[i].task].nch) return "tsqr chunk ref";
                break;
            }
            case ST_GRAM:
            case ST_REDUCE:
            case ST_NN:
            case ST_SUM: {
                const ThinTask* T = (const ThinTask*)(b + s.tasks_off);
                int ntask = s.n;
                if (s.kind != ST_REDUCE) {
                    const ChunkRef* R = (const ChunkRef*)(b + s.refs_off);
                    ntask = 0;
                    for (int i = 0; i < s.n; ++i) ntask = std::max(ntask, R[i].task + 1);
                }
                for (int i = 0; i < ntask; ++i) {
                    const ThinTask& t = T[i];
                    if (t.wx > 128 || t.wy > 128) return "thin width";
                    if (s.tx < 1 || s.tx > 2 || s.ty < 1 || s.ty > 2) return "thin tile grid";
                    if ((s.kind == ST_GRAM && t.wx > 64 * s.tx) || ((s.kind == ST_GRAM || s.kind == ST_NN) && t.wy > 64 * s.ty))
                        return "thin tile grid narrower than a task";
                    if (s.kind == ST_GRAM) {
                        if (!panel("gram X", t.x_off, t.x_ld, t.h, t.wx)) return msg;
                        if (!panel("gram Y", t.y_off, t.y_ld, t.h, t.wy)) return msg;
                        if (!span("gram part", t.part_off, t.part_off + (int64_t)t.nch * t.wx * t.wy - 1, WS)) return msg;
                    } else if (s.kind == ST_REDUCE) {
                        if (t.wx * t.wy > s.w) return "reduce grid";
                        if (!span("reduce part", t.part_off, t.part_off + (int64_t)t.nch * t.wx * t.wy - 1, WS)) return msg;
                        if (!panel("reduce C", t.c_off, t.c_ld, t.wx, t.wy)) return msg;
                        if (t.acc_off >= 0 && !panel("reduce acc", t.acc_off, t.c_ld, t.wx, t.wy)) return msg;
                    } else if (s.kind == ST_NN) {
                        if (t.cond >= IW) return "nn condition slot";
                        if (!panel("nn X", t.x_off, t.x_ld, t.h, t.wx)) return msg;
                        if (!panel("nn C", t.c_off, t.c_ld, t.wx, t.wy)) return msg;
                        if (!panel("nn Y", t.y_off, t.y_ld, t.h, t.wy)) return msg;
                        if (t.x2_off >= 0) {
                            if (t.wx2 < 1 || t.wx2 > 128) return "nn second width";
                            if (!panel("nn X2", t.x2_off, t.x2_ld, t.h, t.wx2)) return msg;
                            if (!panel("nn C2", t.c2_off, t.c2_ld, t.wx2, t.wy)) return msg;
                        }
                    } else {
                        if (t.x_ld < t.h) return "sum ld";
                        if (!span("sum parts", t.x_off, t.x_off + (int64_t)(t.wx - 1) * t.c_ld + (int64_t)(t.wy - 1) * t.x_ld + t.h - 1, WS)) return msg;
                        if (!panel("sum Y", t.y_off, t.y_ld, t.h, t.wy)) return msg;
                    }
                }
                break;
            }
            case ST_ENERGY: {
                const GemmTask* T = (const GemmTask*)(b + s.tasks_off);
                if (!span("energy out", s.off, s.off + s.n - 1, WS)) return msg;
                for (int i = 0; i < s.n; ++i) {
                    const GemmTask& t = T[i];
                    if (t.mat < 0 || t.mat >= (int)P.mats.size()) return "energy matrix index";
                    const MatDesc& M = P.mats[t.mat];
                    const int64_t ld = M.trans ? M.m : M.n;
                    if (t.lda != ld || t.cols > ld || t.a_off % ld + t.cols > ld) return "energy block";
                    if (!span("energy A", t.a_off, t.a_off + (int64_t)(t.rows - 1) * ld + t.cols - 1, M.m * M.n)) return msg;
                }
                break;
            }
            case ST_GRAMX: {
                if (!P.gram || P.mats.size() != 2) return "Gram stage outside a Gram plan";
                const MatDesc& X = P.mats[1];
                const int T = (int)((X.n + 63) / 64);
                const int64_t rows = s.off2, nch = (X.m + rows - 1) / std::max<int64_t>(rows, 1);
                if (rows < 1) return "Gram chunk rows";
                if (!span("Gram partials", s.off, s.off + nch * X.n * X.n - 1, WS)) return msg;
                const GramRef* R = (const GramRef*)(b + s.tasks_off);
                for (int i = 0; i < s.n; ++i)
                    if (R[i].ti < 0 || R[i].ti > R[i].tj || R[i].tj >= T || R[i].chunk < 0 || R[i].chunk >= nch)
                        return "Gram tile ref";
                break;
            }
            case ST_PQR: {
                const TsqrTask* T = (const TsqrTask*)(b + s.tasks_off);
                if (s.w < 1 || s.w > kPanelQrMaxW) return "panel qr width";
                if (s.ordered) {
                    const int* O = (const int*)(b + s.order_off);
                    std::vector<char> seen((size_t)s.n, 0);
                    for (int i = 0; i < s.n; ++i) {
                        if (O[i] < 0 || O[i] >= s.n || seen[(size_t)O[i]]) return "panel qr order";
                        seen[(size_t)O[i]] = 1;
                    }
                }
                for (int i = 0; i < s.n; ++i) {
                    const TsqrTask& t = T[i];
                    if (t.pq_q_off < 0) continue;
                    if (!panel("panel qr P", t.p_off, t.p_ld, t.h, s.w)) return msg;
                    if (!panel("panel qr Q", t.pq_q_off, t.pq_q_ld, t.h, s.w)) return msg;
                    const int64_t p_end = t.p_off + (int64_t)(s.w - 1) * t.p_ld + t.h;
                    const int64_t q_end = t.pq_q_off + (int64_t)(s.w - 1) * t.pq_q_ld + t.h;
                    if (t.pq_q_off < p_end && t.p_off < q_end) return "panel qr Q overlaps P";
                    if (!span("panel qr scratch", t.pq_scr, t.pq_scr + 2LL * s.w * s.w - 1, WS)) return msg;
                    if (s.need_r != 0 && s.need_r != 1 && s.need_r != kPqrSpanOnly) return "panel qr mode";
                    if (s.need_r == 1 && !span("panel qr R", t.r_out, t.r_out + (int64_t)s.w * s.w - 1, WS)) return msg;
                    if (t.cq_flag < 0 || t.cq_flag >= IW) return "panel qr flag slot";
                }
                break;
            }
            case ST_LEAFCHECK: {
                const LeafCheck* T = (const LeafCheck*)(b + s.tasks_off);
                if (s.done_slot < 0 || s.done_slot >= IW || s.step < 1) return "leaf check slot";
                for (int i = 0; i < s.n; ++i)
                    if (T[i].w < 1 || !span("leaf check sigma", T[i].sig_off, T[i].sig_off + T[i].w - 1, WS))
                        return T[i].w < 1 ? "leaf check width" : msg;
                break;
            }
            case ST_ESUM: {
                const EnergySum* T = (const EnergySum*)(b + s.tasks_off);
                if (!span("energy parts", s.off2, s.off2 + std::max(s.w, 1) - 1, WS)) return msg;
                for (int i = 0; i < s.n; ++i) {
                    if (T[i].first < 0 || T[i].count < 1 || T[i].first + T[i].count > s.w) return "energy part range";
                    if (!span("energy sum out", T[i].out, T[i].out, WS)) return msg;
                }
                break;
            }
            case ST_FEAT: {
                if (!span("feature sigma", s.off, s.off + 16LL * s.n - 1, WS)) return msg;
                if (!span("feature energy", s.off2, s.off2 + s.n - 1, WS)) return msg;
                break;
            }
            case ST_CORE: {
                const CoreTask* T = (const CoreTask*)(b + s.tasks_off);
                const bool wide = s.maxdim > kCoreMaxN;
                if (s.maxdim < 1 || s.maxdim > kWideCoreMaxN || (s.with_v && s.maxdim > kCoreMaxV)) return "core size";
                for (int i = 0; i < s.n; ++i) {
                    const CoreTask& t = T[i];
                    const int W = s.pw;
                    if (wide) {
                        if (t.scr_off < 0 || !span("wide core scratch", t.scr_off, t.scr_off + kWideScratch - 1, WS))
                            return "wide core scratch";
                        if (t.energy_off >= 0 || t.v_off >= 0) return "wide core outputs";
                    }
                    if (t.mode == CORE_MERGE) {
                        if (2 * t.kcap > s.maxdim || t.kcap > W) return "merge core exceeds maxdim";
                        if (!span("core s1", t.s1_off, t.s1_off + W - 1, WS)) return msg;
                        if (!span("core s2", t.s2_off, t.s2_off + W - 1, WS)) return msg;
                        if (!panel("core C", t.c_off, t.c_ld, W, W)) return msg;
                        if (!panel("core R", t.r_off, t.r_ld, W, W)) return msg;
                        if (!span("core ranks", std::min(t.rank1, t.rank2), std::max(t.rank1, t.rank2), IW)) return msg;
                        if (!panel("core T", t.t_off, t.t_ld, t.t_ld, t.out_w)) return msg;
                        if (!panel("core X", t.u_off, t.u_ld, t.u_ld, t.out_w)) return msg;
                        if (t.t_ld < W || t.u_ld < W) return "merge outputs too short";
                    } else {
                        if (t.dim > s.maxdim) return "core dim exceeds maxdim";
                        if (!panel("core M", t.m_off, t.m_ld, t.dim, t.dim)) return msg;
                        if (t.rank_in >= IW) return "core rank_in";
                        if (t.u_off >= 0 && !panel("core U", t.u_off, t.u_ld, t.dim, t.out_w)) return msg;
                        if (t.v_off >= 0 && (!s.with_v || !panel("core V", t.v_off, t.v_ld, t.dim, t.out_w))) return msg;
                    }
                    if (!span("core sigma", t.sig_off, t.sig_off + t.out_w - 1, WS)) return msg;
                    if (t.sigall_off >= 0 && (t.mode == CORE_MERGE || !span("core all sigma", t.sigall_off, t.sigall_off + t.dim - 1, WS)))
                        return t.mode == CORE_MERGE ? "all-sigma output of a merge core" : msg;
                    if (t.energy_off >= 0 && (t.energy_off >= WS || t.flag_slot < 0 || t.flag_slot >= IW))
                        return "core energy check";
                    if (t.rank_out >= IW || t.fixed_rank_slot >= IW) return "core rank slot";
                }
                break;
            }
        }
    }
    for (const Stage& s : P.stages)
        if (s.guard >= IW) return "stage guard slot";
    for (int slot : P.reset_slots)
        if (slot < 0 || slot >= IW) return "reset slot";
    if (P.outs.size() != (P.kind == 0 ? (size_t)P.ntree : 0)) return "output count";
    for (size_t mi = 0; mi < P.outs.size(); ++mi) {
        const OutputArgs& o = P.outs[mi];
        const MatDesc& M = P.mats[P.gram ? 1 : mi];
        const int64_t om = M.trans ? M.n : M.m, on = M.trans ? M.m : M.n;   // the input's shape
        const MatDesc& Mt = P.mats[mi];             // the matrix whose trees made the factors
        if (o.m != om || o.n != on || o.k != M.k || o.k > Mt.pw) return "output shape";
        if (!panel("out U", o.u_off, o.u_ld, om, Mt.pw)) return msg;
        if (!panel("out V", o.v_off, o.v_ld, on, Mt.pw)) return msg;
        if (!span("out sigma", o.sig_off, o.sig_off + Mt.pw - 1, WS)) return msg;
        if (!span("out signs", o.sign_off, o.sign_off + M.k - 1, IW)) return msg;
        if (o.rank_slot < 0 || o.rank_slot >= IW) return "out rank slot";
    }
    if (!span("omega", P.omega_off, P.omega_off + P.omega_count - 1, WS)) return msg;
    return "";
}

hsvd_status run_stage(hsvd_plan_st& P, const Stage& s, hipStream_t st) {
    unsigned char* b = (unsigned char*)P.dblob;
    hipError_t e = hipSuccess;
    const int fp32 = P.opt.precision != HSVD_FP64 && !s.a64;
    const int* guard = s.guard >= 0 ? P.iws + s.guard : nullptr;
    switch (s.kind) {
        case ST_GEMM:
            if (s.bf16)
                e = launch_gemm_bf16(s.op, (const void* const*)P.dptrs, P.ws, (const GemmTask*)(b + s.tasks_off),
                                     (const TileRef*)(b + s.refs_off), s.n, s.N, st);
            else if (s.f32)
                e = launch_gemm_f32(s.op, (const void* const*)P.dptrs, P.ws, (const GemmTask*)(b + s.tasks_off),
                                    (const TileRef*)(b + s.refs_off), s.n, s.N, st);
            else
                e = launch_gemm(s.op, fp32, (const void* const*)P.dptrs, P.ws, (const GemmTask*)(b + s.tasks_off),
                                (const TileRef*)(b + s.refs_off), s.n, s.N, st, guard, s.e_part);
            break;
        case ST_CQ1:
        case ST_CQ2:
            e = launch_cholqr(s.kind == ST_CQ1 ? 1 : 2, P.ws, P.iws, (const TsqrTask*)(b + s.tasks_off),
                              (const ChunkRef*)(b + s.refs_off), s.n, s.w, s.ch, st);
            break;
        case ST_GRAMX: {
            const MatDesc& X = P.mats[1];
            e = launch_gram_xtx(P.opt.precision != HSVD_FP64, (const void* const*)P.dptrs, 1, X.m, X.n, s.off2, P.ws,
                                s.off, (const GramRef*)(b + s.tasks_off), s.n, st);
            break;
        }
        case ST_PQR:
            e = launch_panel_qr(P.ws, P.iws, (const TsqrTask*)(b + s.tasks_off), s.n, s.w, s.need_r, st, guard,
                                s.ordered ? (const int*)(b + s.order_off) : nullptr);
            break;
        case ST_TSQR_F:
            e = launch_tsqr_factor(P.ws, P.iws, (const TsqrTask*)(b + s.tasks_off),
                                   (const ChunkRef*)(b + s.refs_off), s.n, s.w, s.ch, st, guard);
            break;
        case ST_TSQR_A:
            e = launch_tsqr_apply(P.ws, P.iws, (const TsqrTask*)(b + s.tsqr_off),
                                  (const ApplyTask*)(b + s.tasks_off),
                                  (const ChunkRef*)(b + s.refs_off), s.n, s.w, s.ch, s.c, st, guard);
            break;
        case ST_GRAM:
            e = launch_thin_gram(P.ws, (const ThinTask*)(b + s.tasks_off),
                                 (const ChunkRef*)(b + s.refs_off), s.n, P.thin_ch, st, s.tx, s.ty);
            break;
        case ST_REDUCE:
            e = launch_thin_reduce(P.ws, (const ThinTask*)(b + s.tasks_off), s.n, s.w, st);
            break;
        case ST_NN:
            e = launch_thin_nn(P.ws, P.iws, (const ThinTask*)(b + s.tasks_off),
                               (const ChunkRef*)(b + s.refs_off), s.n, P.thin_ch, st, s.ty);
            break;
        case ST_SUM:
            e = launch_thin_sum(P.ws, (const ThinTask*)(b + s.tasks_off),
                                (const ChunkRef*)(b + s.refs_off), s.n, P.thin_ch, st);
            break;
        case ST_CORE:
            e = launch_core(P.ws, P.iws, (const CoreTask*)(b + s.tasks_off), s.n, s.maxdim,
                            P.opt.max_sweeps, P.flags, s.with_v, st, guard);
            break;
        case ST_LEAFCHECK:
            e = launch_leaf_check(P.ws, P.iws, (const LeafCheck*)(b + s.tasks_off), s.n, s.step, s.done_slot,
                                  guard, st);
            break;
        case ST_ENERGY:
            e = launch_block_energy((const void* const*)P.dptrs, fp32, (const GemmTask*)(b + s.tasks_off),
                                    s.n, P.ws, s.off, st);
            break;
        case ST_ESUM:
            e = launch_energy_sum(P.ws, s.off2, (const EnergySum*)(b + s.tasks_off), s.n, st);
            break;
        case ST_FEAT:
            e = launch_block_features(P.ws, s.off, s.off2, s.n, (float*)P.host_ptrs[1], st);
            break;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return HSVD_OK;
}

}  // namespace

extern "C" {

hsvd_status hsvd_default_options(hsvd_options* opt) {
    if (!opt) return fail(HSVD_ERR_INVALID, "opt is NULL");
    opt->precision = HSVD_FP64;
    opt->rule = HSVD_RULE_GAMMA;
    opt->oversample = 14;
    opt->power_steps = -1;
    opt->refine_steps = 0;
    opt->max_sweeps = 40;
    opt->seed = 0;
    opt->refine_eps = 0.0;
    opt->graph = 1;
    opt->order = HSVD_ORDER_AUTO;
    opt->thin_rows = 0;
    opt->merge_qr = 0;
    opt->leaf_qr = 0;
    opt->autotune = 0;
    return HSVD_OK;
}

// Bytes of the arena and the int arena as hsvd_set_workspace lays them out.
static size_t workspace_need(const hsvd_plan_st& P) {
    const size_t ws_bytes = sizeof(double) * (size_t)std::max<int64_t>(P.ws_elems, 32);
    return (ws_bytes + 255) / 256 * 256 + sizeof(int) * (size_t)std::max(P.iws_elems, 1);
}

static hsvd_status execute_impl(hsvd_plan_st& P, const void* const* A, void* const* U, void* const* S,
                                void* const* Vt, hipStream_t stream);
static hsvd_status plan_impl(hsvd_plan_t* out, int32_t count, const int64_t* ms, const int64_t* ns,
                             const int32_t* ps, const int32_t* qs, const int32_t* ks, double tol,
                             const hsvd_options* opt, size_t* check_only, const int32_t* leaf_width = nullptr,
                             int kind = 0, bool host_only = false);

// Sketch width of a leaf from the network's prediction y = log2(rank): ceil(2^y) plus a
// margin of 8 columns, rounded up to a multiple of 8 (few width classes, one pipeline
// each), between 8 and the largest width the leaf kernels take (and the block's sides).
static int learned_width(float y, int64_t rows, int64_t cols) {
    const int lmax = (int)std::min<int64_t>(kTsqrMaxW, std::min(rows, cols));
    if (!std::isfinite(y) || y > 16.0f) return lmax;
    const double k = std::ceil(std::exp2((double)y));
    const int w = (int)(std::ceil((k + 8.0) / 8.0) * 8.0);
    return std::max(1, std::min(std::max(w, 8), lmax));
}

// The learned path of an execute: features and prediction on the device, widths on the
// host (one read-back), a width plan (rebuilt only when the widths change), then the
// tolerance rule judges each leaf: a leaf whose sketch missed more than tol^2 of its
// block's energy doubles its width and the call runs again (at most 3 times); if a leaf
// still misses, the plain plan (widths k + oversample) computes the result instead.
static hsvd_status learned_execute(hsvd_plan_st& P, const void* A, void* U, void* S, void* Vt,
                                   hipStream_t stream) {
    const MatDesc& M = P.mats[0];
    const int nb = M.p * M.q;
    void* f = P.rm_feat;
    hsvd_status st = execute_impl(*P.rm_features, &A, &f, &f, &f, stream);
    if (st != HSVD_OK) return st;
    hipError_t e = launch_mlp_predict(P.rm_params, P.rm_feat, nb, P.rm_pred, stream);
    std::vector<float> pred((size_t)nb);
    if (e == hipSuccess) e = hipMemcpyAsync(pred.data(), P.rm_pred, sizeof(float) * nb, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "rank prediction");
    std::vector<int> widths((size_t)nb);
    for (int i = 0; i < M.p; ++i)
        for (int j = 0; j < M.q; ++j)
            widths[(size_t)i * M.q + j] = learned_width(pred[(size_t)i * M.q + j], M.brow(i), M.bcol(j));
    P.rm_refits = 0;
    P.rm_plain = 0;
    for (;;) {
        if (!P.rm_wplan || widths != P.rm_widths) {
            if (P.rm_wplan) hsvd_destroy(P.rm_wplan);
            P.rm_wplan = nullptr;
            int64_t m = M.m, n = M.n;
            int32_t p = M.p, q = M.q, k = M.k;
            st = plan_impl(&P.rm_wplan, 1, &m, &n, &p, &q, &k, P.tol, &P.opt, nullptr, widths.data(), 0, false);
            if (st != HSVD_OK) return st;
            P.rm_widths = widths;
        }
        st = execute_impl(*P.rm_wplan, &A, &U, &S, &Vt, stream);
        if (st != HSVD_OK) return st;
        P.rm_ran = P.rm_wplan;
        std::vector<int32_t> fb((size_t)nb);
        st = hsvd_get_leaf_info(P.rm_wplan, nullptr, fb.data(), nb);
        if (st != HSVD_OK) return st;
        bool missed = false, grow = false;
        for (int b = 0; b < nb; ++b) {
            if (!fb[b]) continue;
            missed = true;
            const int lim = learned_width(1e9f, M.brow(b / M.q), M.bcol(b % M.q));
            if (widths[b] < lim) {
                widths[b] = std::min(2 * widths[b], lim);
                grow = true;
            }
        }
        if (!missed) return HSVD_OK;
        if (!grow || P.rm_refits == 3) break;
        ++P.rm_refits;
    }
    P.rm_plain = 1;
    P.rm_ran = &P;
    return execute_impl(P, &A, &U, &S, &Vt, stream);
}

// Kernel attributes every plan may need, set before any launch could be captured.
static hipError_t prepare_launches() {
    hipError_t e = prepare_core_launches();
    if (e == hipSuccess) e = prepare_panel_qr_launches();
    if (e == hipSuccess) e = prepare_gemm_bf16_launches();
    if (e == hipSuccess) e = prepare_gemm_f32_launches();
    return e;
}

// ---------------------------------------------------------------- plan-time autotuning
// The tunables (thin_rows, merge_qr) change how the work is cut into launches, never
// the arithmetic of a result's entries beyond the order of float64 sums.  Candidates are
// timed as whole executes on a Gaussian input of the plan's shapes; the choice is kept
// per (device, plan kind, options, shapes) for the process and, with HSVD_TUNE_CACHE
// set, in that file (one line per key: hash, thin_rows, merge_qr, leaf_qr, median ms).
namespace {
std::mutex g_tune_mu;
std::map<uint64_t, Tuning> g_tune;
bool g_tune_file_read = false;

uint64_t tune_key(int32_t count, const int64_t* ms, const int64_t* ns, const int32_t* ps, const int32_t* qs,
                  const int32_t* ks, double tol, const hsvd_options& o, int kind) {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
    std::string k = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
    char buf[256];
    snprintf(buf, sizeof buf, "|%d|%d,%d,%d,%d,%d,%d,%d,%.17g", kind, o.precision, o.rule, o.oversample,
             o.power_steps, o.refine_steps, o.order, o.graph, tol);
    k += buf;
    for (int i = 0; i < count; ++i) {
        snprintf(buf, sizeof buf, "|%lldx%lld:%dx%d:%d", (long long)ms[i], (long long)ns[i], ps[i], qs[i], ks[i]);
        k += buf;
    }
    uint64_t h = 1469598103934665603ull;          // FNV-1a, 64 bit
    for (unsigned char c : k) { h ^= c; h *= 1099511628211ull; }
    return h;
}

void tune_file_read() {
    const char* path = std::getenv("HSVD_TUNE_CACHE");
    if (!path || g_tune_file_read) return;
    g_tune_file_read = true;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string hex;
        Tuning t{};
        if (!(is >> hex >> t.thin_rows >> t.merge_qr >> t.leaf_qr >> t.ms)) continue;
        if (t.thin_rows != 0 && (t.thin_rows < 64 || t.thin_rows > 1024 || t.thin_rows % 64)) continue;
        if (t.merge_qr < 0 || t.merge_qr > 3 || t.leaf_qr < 0 || t.leaf_qr > 2) continue;
        g_tune[std::stoull(hex, nullptr, 16)] = t;
    }
}

void tune_file_append(uint64_t key, const Tuning& t) {
    const char* path = std::getenv("HSVD_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    char buf[96];
    snprintf(buf, sizeof buf, "%016llx %d %d %d %.4f\n", (unsigned long long)key, t.thin_rows, t.merge_qr,
             t.leaf_qr, t.ms);
    f << buf;
}
}  // namespace

static hsvd_status autotune(int32_t count, const int64_t* ms, const int64_t* ns, const int32_t* ps,
                            const int32_t* qs, const int32_t* ks, double tol, const hsvd_options& o, int kind,
                            Tuning* out) {
    const uint64_t key = tune_key(count, ms, ns, ps, qs, ks, tol, o, kind);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_file_read();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            return HSVD_OK;
        }
    }
    // a Gaussian input and outputs for every matrix, in the plan's element type
    const bool f32 = o.precision != HSVD_FP64;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const int nmat = count;
    std::vector<void*> bufs;
    auto release = [&]() { for (void* b : bufs) hipFree(b); bufs.clear(); };
    std::vector<const void*> A(nmat);
    std::vector<void*> U(nmat), S(nmat), V(nmat);
    hipError_t e = hipSuccess;
    for (int i = 0; i < nmat && e == hipSuccess; ++i) {
        void *a = nullptr, *u = nullptr, *sv = nullptr, *v = nullptr;
        e = hipMalloc(&a, es * (size_t)ms[i] * ns[i]);
        if (e == hipSuccess) bufs.push_back(a);
        if (e == hipSuccess && (e = hipMalloc(&u, es * (size_t)ms[i] * ks[i])) == hipSuccess) bufs.push_back(u);
        if (e == hipSuccess && (e = hipMalloc(&sv, es * (size_t)ks[i])) == hipSuccess) bufs.push_back(sv);
        if (e == hipSuccess && (e = hipMalloc(&v, es * (size_t)ks[i] * ns[i])) == hipSuccess) bufs.push_back(v);
        if (e == hipSuccess)
            e = f32 ? launch_gaussian_f32((float*)a, ms[i] * ns[i], 0x7417ull + (uint64_t)i, 0)
                    : launch_gaussian((double*)a, ms[i] * ns[i], 0x7417ull + (uint64_t)i, 0);
        A[i] = a; U[i] = u; S[i] = sv; V[i] = v;
    }
    hipStream_t st = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release();
        if (st) hipStreamDestroy(st);
        return hip_fail(e, "autotune set-up");
    }
    hipEvent_t ev[4] = {};
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    // median of three timed executes after one warm-up; a candidate the plan builder or
    // the device rejects scores +inf
    auto run = [&](int thin_rows, int merge_qr, int leaf_qr) -> float {
        hsvd_options c = o;
        c.autotune = 0;
        c.thin_rows = thin_rows;
        c.merge_qr = merge_qr;
        c.leaf_qr = leaf_qr;
        hsvd_plan_t cp = nullptr;
        if (plan_impl(&cp, count, ms, ns, ps, qs, ks, tol, &c, nullptr, nullptr, kind, false) != HSVD_OK)
            return INFINITY;
        auto exec = [&]() -> bool {
            if (nmat == 1)
                return hsvd_execute(cp, A[0], U[0], S[0], V[0], st) == HSVD_OK;
            return hsvd_execute_batched(cp, A.data(), U.data(), S.data(), V.data(), st) == HSVD_OK;
        };
        float t[3] = {INFINITY, INFINITY, INFINITY};
        bool ok = exec() && hipStreamSynchronize(st) == hipSuccess;
        for (int r = 0; r < 3 && ok; ++r) {
            ok = hipEventRecord(ev[0], st) == hipSuccess && exec() && hipEventRecord(ev[1], st) == hipSuccess &&
                 hipEventSynchronize(ev[1]) == hipSuccess && hipEventElapsedTime(&t[r], ev[0], ev[1]) == hipSuccess;
        }
        hsvd_destroy(cp);
        if (!ok) return INFINITY;
        std::sort(t, t + 3);
        return t[1];
    };
    Tuning best{};
    best.ms = (e == hipSuccess) ? run(0, 0, 0) : INFINITY;
    for (int lq : {1, 2}) {
        const float x = run(0, 0, lq);
        if (x < best.ms) { best.ms = x; best.leaf_qr = lq; }
    }
    for (int tr : {256, 512}) {
        const float x = run(tr, 0, best.leaf_qr);
        if (x < best.ms) { best.ms = x; best.thin_rows = tr; }
    }
    for (int bit : {1, 2}) {
        const int mq = best.merge_qr | bit;
        const float x = run(best.thin_rows, mq, best.leaf_qr);
        if (x < best.ms) { best.ms = x; best.merge_qr = mq; }
    }
    for (auto& x : ev)
        if (x) hipEventDestroy(x);
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
    release();
    if (!std::isfinite(best.ms)) return fail(HSVD_ERR_HIP, "autotune: no candidate ran");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
        tune_file_append(key, best);
    }
    *out = best;
    return HSVD_OK;
}

static hsvd_status plan_impl(hsvd_plan_t* out, int32_t count, const int64_t* ms, const int64_t* ns,
                             const int32_t* ps, const int32_t* qs, const int32_t* ks, double tol,
                             const hsvd_options* opt, size_t* check_only,
                             const int32_t* leaf_width, int kind, bool host_only) {
    if (!out && !check_only) return fail(HSVD_ERR_INVALID, "out is NULL");
    if (out) *out = nullptr;
    if (count < 1) return fail(HSVD_ERR_INVALID, "count must be >= 1");
    if (!ms || !ns || !ps || !qs || !ks) return fail(HSVD_ERR_INVALID, "NULL shape array");
    if (count > 65535) return fail(HSVD_ERR_UNSUPPORTED, "more than 65535 matrices in one plan");
    for (int i = 0; i < count; ++i) {
        const int64_t m = ms[i], n = ns[i];
        const int32_t p = ps[i], q = qs[i], k = ks[i];
        const std::string at = count > 1 ? " (matrix " + std::to_string(i) + ")" : "";
        if (m < 1 || n < 1) return fail(HSVD_ERR_INVALID, "m and n must be >= 1" + at);
        if (p < 1 || p > (kind == 2 ? n : m))       // a Gram plan's grid is over the n x n X^T X
            return fail(HSVD_ERR_INVALID, std::string(kind == 2 ? "need 1 <= p <= n" : "need 1 <= p <= m") + at);
        if (q < 1 || q > n) return fail(HSVD_ERR_INVALID, "need 1 <= q <= n" + at);
        if (k < 1 || k > std::min(m, n)) return fail(HSVD_ERR_INVALID, "need 1 <= k <= min(m, n)" + at);
        if (m > (int64_t)1 << 30 || n > (int64_t)1 << 30)
            return fail(HSVD_ERR_UNSUPPORTED, "m and n must be below 2^30" + at);
        if (k > kMaxRank)
            return fail(HSVD_ERR_UNSUPPORTED, "k > " + std::to_string(kMaxRank) + " is not supported by this build" + at);
    }
    if (!(tol >= 0.0 && tol < 1.0)) return fail(HSVD_ERR_INVALID, "need 0 <= tol < 1");
    hsvd_options o;
    hsvd_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != HSVD_FP64 && o.precision != HSVD_FP32 && o.precision != HSVD_MIXED_BF16)
        return fail(HSVD_ERR_INVALID, "unknown precision");
    if (o.rule != HSVD_RULE_GAMMA && o.rule != HSVD_RULE_FROB)
        return fail(HSVD_ERR_INVALID, "unknown rule");
    if (o.oversample < 0 || o.power_steps < -1 || o.refine_steps < 0 || o.max_sweeps < 1)
        return fail(HSVD_ERR_INVALID, "negative option");
    if (o.power_steps > 64) return fail(HSVD_ERR_INVALID, "power_steps above 64");
    if (!(o.refine_eps >= 0.0)) return fail(HSVD_ERR_INVALID, "need refine_eps >= 0");
    if (o.graph != 0 && o.graph != 1) return fail(HSVD_ERR_INVALID, "graph must be 0 or 1");
    if (o.order < HSVD_ORDER_AUTO || o.order > HSVD_ORDER_COLS_LAST) return fail(HSVD_ERR_INVALID, "unknown order");
    if (o.thin_rows != 0 && (o.thin_rows < 64 || o.thin_rows > 1024 || o.thin_rows % 64))
        return fail(HSVD_ERR_INVALID, "thin_rows must be 0 or a multiple of 64 in 64..1024");
    if (o.merge_qr < 0 || o.merge_qr > 3) return fail(HSVD_ERR_INVALID, "merge_qr must be 0..3");
    if (o.leaf_qr < 0 || o.leaf_qr > 2) return fail(HSVD_ERR_INVALID, "leaf_qr must be 0..2");
    if (o.autotune != 0 && o.autotune != 1) return fail(HSVD_ERR_INVALID, "autotune must be 0 or 1");

    Tuning tuned{};
    if (o.autotune && !check_only && !host_only && kind != 1) {
        hsvd_status st = autotune(count, ms, ns, ps, qs, ks, tol, o, kind, &tuned);
        if (st != HSVD_OK) return st;
        o.thin_rows = tuned.thin_rows;
        o.merge_qr = tuned.merge_qr;
        o.leaf_qr = tuned.leaf_qr;
    }
    hsvd_plan_st* P = new (std::nothrow) hsvd_plan_st();
    if (!P) return fail(HSVD_ERR_ALLOC, "host allocation failed");
    P->tol = tol;
    P->opt = o;
    P->thin_ch = o.thin_rows ? o.thin_rows : THIN_CH;
    P->merge_qr = o.merge_qr;
    P->leaf_qr = o.leaf_qr;
    P->tuned = (o.autotune && !check_only && !host_only && kind != 1) ? 1 : 0;
    P->tuned_ms = tuned.ms;
    // merge order: column slabs last (the plan works on the transpose) when asked, or
    // automatically for a single short-fat matrix so that the last tree and the final
    // projection run on the shorter side; learned-width and feature plans keep the
    // order of Algorithm 1
    const bool gram = kind == 2;                 // hsvd_plan_gram: the trees decompose X^T X
    if (gram) {
        kind = 0;
        if (count != 1 || leaf_width || o.precision == HSVD_MIXED_BF16) {
            delete P;
            return fail(HSVD_ERR_UNSUPPORTED, "Gram plans take one float64 or float32 matrix");
        }
    }
    P->gram = gram;
    P->trans = !gram && (o.order == HSVD_ORDER_COLS_LAST ||
                         (o.order == HSVD_ORDER_AUTO && count == 1 && ms[0] < ns[0] && !leaf_width && kind == 0));
    if (P->trans && (leaf_width || kind != 0)) {
        delete P;
        return fail(HSVD_ERR_UNSUPPORTED, "width and feature plans merge row slabs last");
    }
    int kmax = 0, lwant = 1;
    int64_t bmin = INT64_MAX;
    const int nmat = gram ? 2 : count;
    for (int i = 0; i < nmat; ++i) {
        MatDesc M;
        M.trans = P->trans;
        if (gram && i == 0) { M.m = ns[0]; M.n = ns[0]; M.p = ps[0]; M.q = qs[0]; }      // G = X^T X
        else if (gram) { M.m = ms[0]; M.n = ns[0]; M.q = qs[0];                            // X (projection blocks)
                         M.p = (int)std::max<int64_t>(1, std::min<int64_t>(ms[0], (ms[0] + 2047) / 2048)); }
        else if (!P->trans) { M.m = ms[i]; M.n = ns[i]; M.p = ps[i]; M.q = qs[i]; }
        else { M.m = ns[i]; M.n = ms[i]; M.p = qs[i]; M.q = ps[i]; }
        M.k = ks[gram ? 0 : i];
        M.rs.resize(M.p + 1);
        M.cs.resize(M.q + 1);
        for (int r = 0; r <= M.p; ++r) M.rs[r] = (M.m / M.p) * r + std::min<int64_t>(r, M.m % M.p);
        for (int c = 0; c <= M.q; ++c) M.cs[c] = (M.n / M.q) * c + std::min<int64_t>(c, M.n % M.q);
        if (!(gram && i == 1)) bmin = std::min(bmin, std::min(M.m / M.p, M.n / M.q));
        kmax = std::max(kmax, M.k);
        lwant = std::max(lwant, M.k + o.oversample);
        P->mats.push_back(std::move(M));
    }
    P->ntree = gram ? 1 : (int)P->mats.size();
    // one panel width for the whole batch (per-matrix rank caps stay in the tasks);
    // the sketch width of a single matrix (a batched plan's matrices take their own,
    // batch_width)
    P->W = kmax;
    P->L = (int)std::min<int64_t>(lwant, bmin);
    if (P->L < 1) P->L = 1;
    if (P->L > kTsqrMaxW) P->L = kTsqrMaxW;
    // power_steps = -1: float64 plans iterate their leaves until converged (at most
    // kLeafPowerCap steps); float32-storage and mixed plans, whose inputs carry their
    // own rounding, and width plans take one step
    const bool converge = o.power_steps < 0 && o.precision == HSVD_FP64 && !leaf_width && kind == 0;
    P->g = 2 + (o.power_steps < 0 ? 1 : o.power_steps);
    if (converge) P->leaf_cap = kLeafPowerCap;
    P->kind = kind;
    if (leaf_width) {
        const MatDesc& M = P->mats[0];
        int wmax = 1;
        for (int b = 0; b < M.p * M.q; ++b) {
            const int w = leaf_width[b];
            if (w < 1 || w > kTsqrMaxW) {
                delete P;
                return fail(HSVD_ERR_INVALID, "leaf widths must be in 1.." + std::to_string(kTsqrMaxW));
            }
            wmax = std::max(wmax, w);
        }
        P->leaf_width.assign(leaf_width, leaf_width + M.p * M.q);
        P->L = wmax;
    }

    if (kind == 1) build_features(*P);
    else build_plan(*P);
    P->reset_off = P->put(P->reset_slots);
    const std::string verr = validate_plan(*P);
    if (!verr.empty()) { delete P; return fail(HSVD_ERR_INVALID, "plan validation: " + verr); }
    if (check_only) {
        *check_only = sizeof(double) * (size_t)P->ws_elems;
        delete P;
        return HSVD_OK;
    }

    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) { delete P; return hip_fail(e, "hipGetDevice"); }
    if (host_only) {                  // the caller places the device state itself
        *out = P;
        return HSVD_OK;
    }
    e = hipMalloc(&P->ws, sizeof(double) * (size_t)std::max<int64_t>(P->ws_elems, 32));
    if (e != hipSuccess) { delete P; return fail(HSVD_ERR_ALLOC, "workspace allocation failed"); }
    e = hipMalloc(&P->iws, sizeof(int) * (size_t)std::max(P->iws_elems, 1));
    if (e == hipSuccess) e = hipMalloc(&P->flags, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = hipMalloc(&P->dblob, std::max<size_t>(P->blob.size(), 256));
    if (e == hipSuccess) e = hipMalloc((void**)&P->dptrs, sizeof(void*) * 4 * P->mats.size());
    if (e != hipSuccess) { hsvd_destroy(P); return fail(HSVD_ERR_ALLOC, "allocation failed"); }
    e = hipMemcpy(P->dblob, P->blob.data(), P->blob.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(P->iws, 0, sizeof(int) * (size_t)std::max(P->iws_elems, 1));
    if (e == hipSuccess) e = hipMemset(P->flags, 0, sizeof(unsigned) * 4);
    if (e == hipSuccess) e = hipMemset(P->ws, 0, sizeof(double) * (size_t)P->ws_elems);
    if (e == hipSuccess) e = hipMemset(P->dptrs, 0, sizeof(void*) * 4 * P->mats.size());
    for (auto& c : P->ws_init)
        if (e == hipSuccess)
            e = hipMemcpy(P->ws + c.first, c.second.data(), c.second.size() * sizeof(double),
                          hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_gaussian(P->ws + P->omega_off, P->omega_count, o.seed, 0);
    if (e == hipSuccess) e = prepare_launches();
    // streams and events of the concurrent leaf classes (default priority)
    if (e == hipSuccess && P->nbranch > 0) {
        e = hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming);
        for (int b = 0; b < P->nbranch && e == hipSuccess; ++b) {
            hipStream_t bs = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
            if (e == hipSuccess) P->bstreams.push_back(bs);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) P->join_ev.push_back(ev);
        }
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { hsvd_destroy(P); return hip_fail(e, "plan initialisation"); }
    *out = P;
    return HSVD_OK;
}

hsvd_status hsvd_plan_ex(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                         double tol, const hsvd_options* opt) {
    return plan_impl(out, 1, &m, &n, &p, &q, &k, tol, opt, nullptr);
}

hsvd_status hsvd_plan_batched(hsvd_plan_t* out, int32_t count, const int64_t* m, const int64_t* n,
                              const int32_t* p, const int32_t* q, const int32_t* k, double tol,
                              const hsvd_options* opt) {
    return plan_impl(out, count, m, n, p, q, k, tol, opt, nullptr);
}

hsvd_status hsvd_debug_plan_check(int64_t m, int64_t n, int32_t p, int32_t q, int32_t k, double tol,
                                  const hsvd_options* opt, size_t* workspace_bytes) {
    size_t bytes = 0;
    hsvd_status st = plan_impl(nullptr, 1, &m, &n, &p, &q, &k, tol, opt, &bytes);
    if (workspace_bytes) *workspace_bytes = bytes;
    return st;
}

hsvd_status hsvd_plan_widths(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                             double tol, const hsvd_options* opt, const int32_t* leaf_width) {
    if (!leaf_width) return fail(HSVD_ERR_INVALID, "leaf_width is NULL");
    return plan_impl(out, 1, &m, &n, &p, &q, &k, tol, opt, nullptr, leaf_width, 0);
}

hsvd_status hsvd_features_plan(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q,
                               int32_t precision, uint64_t seed) {
    hsvd_options o;
    hsvd_default_options(&o);
    o.precision = precision;
    o.seed = seed;
    if (precision == HSVD_MIXED_BF16) return fail(HSVD_ERR_INVALID, "feature plans take FP64 or FP32");
    const int32_t k = 1;
    return plan_impl(out, 1, &m, &n, &p, &q, &k, 0.0, &o, nullptr, nullptr, 1);
}

hsvd_status hsvd_debug_plan_check_batched(int32_t count, const int64_t* m, const int64_t* n,
                                          const int32_t* p, const int32_t* q, const int32_t* k,
                                          double tol, const hsvd_options* opt, size_t* workspace_bytes) {
    size_t bytes = 0;
    hsvd_status st = plan_impl(nullptr, count, m, n, p, q, k, tol, opt, &bytes);
    if (workspace_bytes) *workspace_bytes = bytes;
    return st;
}

hsvd_status hsvd_plan_gram(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                           double tol, const hsvd_options* opt) {
    return plan_impl(out, 1, &m, &n, &p, &q, &k, tol, opt, nullptr, nullptr, 2);
}

hsvd_status hsvd_plan(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                      double tol) {
    return hsvd_plan_ex(out, m, n, p, q, k, tol, nullptr);
}

// Every launch of one execute (a plan not stopped on refine_eps), in order, on `stream`.
// Stages [begin, end) on `stream`; a run of leaf-class stages (branch > 0) forks: each
// class runs in order on its own stream after an event recorded on `stream`, and
// `stream` waits for every class before the stage after the run (under graph capture
// the classes become parallel branches of the graph).
static hsvd_status run_stages(hsvd_plan_st& P, size_t begin, size_t end, hipStream_t stream) {
    for (size_t i = begin; i < end;) {
        if (P.stages[i].branch == 0 || P.bstreams.empty()) {
            hsvd_status st = run_stage(P, P.stages[i], stream);
            if (st != HSVD_OK) return st;
            ++i;
            continue;
        }
        size_t j = i;
        while (j < end && P.stages[j].branch > 0) ++j;
        hipError_t e = hipEventRecord(P.fork_ev, stream);
        if (e != hipSuccess) return hip_fail(e, "fork");
        for (int b = 1; b <= P.nbranch; ++b) {
            hipStream_t bs = P.bstreams[(size_t)b - 1];
            if ((e = hipStreamWaitEvent(bs, P.fork_ev, 0)) != hipSuccess) return hip_fail(e, "fork");
            for (size_t k = i; k < j; ++k)
                if (P.stages[k].branch == b) {
                    hsvd_status st = run_stage(P, P.stages[k], bs);
                    if (st != HSVD_OK) return st;
                }
            if ((e = hipEventRecord(P.join_ev[(size_t)b - 1], bs)) != hipSuccess) return hip_fail(e, "join");
            if ((e = hipStreamWaitEvent(stream, P.join_ev[(size_t)b - 1], 0)) != hipSuccess) return hip_fail(e, "join");
        }
        i = j;
    }
    return HSVD_OK;
}

static hsvd_status enqueue_all(hsvd_plan_st& P, hipStream_t stream) {
    hipError_t e = launch_reset_state(P.flags, P.iws, (const int*)((unsigned char*)P.dblob + P.reset_off),
                                      (int)P.reset_slots.size(), stream);
    if (e != hipSuccess) return hip_fail(e, "state reset");
    hsvd_status st0 = run_stages(P, 0, P.stages.size(), stream);
    if (st0 != HSVD_OK) return st0;
    e = launch_output(P.opt.precision != HSVD_FP64, P.ws, P.iws,
                      (const OutputArgs*)((unsigned char*)P.dblob + P.outs_off), (int)P.outs.size(), P.kmax, P.mmax,
                      P.nmax, (void* const*)P.dptrs, stream);
    if (e != hipSuccess) return hip_fail(e, "output launch");
    return HSVD_OK;
}

static hsvd_status execute_impl(hsvd_plan_st& P, const void* const* A, void* const* U, void* const* S,
                                void* const* Vt, hipStream_t stream) {
    const size_t cnt = P.mats.size();
    std::vector<void*> tab(4 * cnt);
    for (size_t i = 0; i < cnt; ++i) {
        if (!A[i] || !U[i] || !S[i] || !Vt[i]) return fail(HSVD_ERR_INVALID, "NULL data pointer");
        tab[4 * i] = const_cast<void*>(A[i]);
        tab[4 * i + 1] = U[i];
        tab[4 * i + 2] = S[i];
        tab[4 * i + 3] = Vt[i];
    }
    hipError_t e = hipSuccess;
    if (tab != P.host_ptrs) {
        // the table is read by the launches of earlier executes on this stream:
        // replace it only once they are done (then the copy is stream-ordered)
        if (P.executed && (e = hipStreamSynchronize(P.last_stream)) != hipSuccess)
            return hip_fail(e, "pointer table");
        e = hipMemcpyAsync(P.dptrs, tab.data(), sizeof(void*) * tab.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "pointer table");
        P.host_ptrs = tab;
    }
    const bool prof = P.profiling && P.events.size() == P.stages.size() + 2;
    if (P.opt.graph && P.seg_end.empty() && !prof) {
        if (!P.gexec) {
            // capture on a stream of the plan's own (the caller's may be the null
            // stream, which cannot be captured); nothing runs during the capture
            if (!P.cap_stream && (e = hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "capture stream");
            if ((e = hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            hsvd_status st = enqueue_all(P, P.cap_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(P.cap_stream, &g);
            if (st != HSVD_OK) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            P.graph = g;
            if ((e = hipGraphInstantiate(&P.gexec, P.graph, nullptr, nullptr, 0)) != hipSuccess) {
                P.gexec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
        }
        if ((e = hipGraphLaunch(P.gexec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        P.last_stream = stream;
        P.executed = true;
        return HSVD_OK;
    }
    e = launch_reset_state(P.flags, P.iws, (const int*)((unsigned char*)P.dblob + P.reset_off),
                           (int)P.reset_slots.size(), stream);
    if (e != hipSuccess) return hip_fail(e, "state reset");
    if (prof && (e = hipEventRecord(P.events[0], stream)) != hipSuccess) return hip_fail(e, "event");
    size_t outs_off = P.outs_off;
    if (P.seg_end.empty() && !prof) {
        hsvd_status st = run_stages(P, 0, P.stages.size(), stream);
        if (st != HSVD_OK) return st;
    } else if (P.seg_end.empty()) {                // per-launch events: one stream, in order
        for (size_t i = 0; i < P.stages.size(); ++i) {
            hsvd_status st = run_stage(P, P.stages[i], stream);
            if (st != HSVD_OK) return st;
            if (prof && (e = hipEventRecord(P.events[i + 1], stream)) != hipSuccess) return hip_fail(e, "event");
        }
    } else {
        // Algorithm 2 until the singular values change by at most refine_eps (relative,
        // 2-norm) between two iterations, at most refine_steps iterations: one 4-byte
        // read-back and host wait per check (the decision itself is taken on the device)
        const size_t nseg = P.seg_end.size();
        size_t i = 0, used = nseg;
        for (size_t t = 0; t < nseg; ++t) {
            hsvd_status st = run_stages(P, i, P.seg_end[t], stream);
            if (st != HSVD_OK) return st;
            i = P.seg_end[t];
            if (t + 1 == nseg) continue;
            e = launch_refine_check(P.ws, P.iws, (const RefineCheck*)((unsigned char*)P.dblob + P.check_off[t]),
                                    P.ntree, P.opt.refine_eps, P.check_slot, stream);
            int done = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&done, P.iws + P.check_slot, sizeof(int), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "refinement check");
            if (done) { used = t + 1; break; }
        }
        outs_off = P.step_outs_off[used - 1];
        P.rank_slots = P.step_rank_slots[used - 1];
        P.refine_done = (int)used;
    }
    e = launch_output(P.opt.precision != HSVD_FP64, P.ws, P.iws,
                      (const OutputArgs*)((unsigned char*)P.dblob + outs_off), (int)P.outs.size(), P.kmax, P.mmax,
                      P.nmax, (void* const*)P.dptrs, stream);
    if (e != hipSuccess) return hip_fail(e, "output launch");
    if (prof && (e = hipEventRecord(P.events.back(), stream)) != hipSuccess) return hip_fail(e, "event");
    P.last_stream = stream;
    P.executed = true;
    return HSVD_OK;
}

hsvd_status hsvd_execute(hsvd_plan_t plan, const void* A, void* U, void* S, void* Vt,
                         hipStream_t stream) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (plan->kind != 0) return fail(HSVD_ERR_INVALID, "feature plan: use hsvd_features_execute");
    if (plan->gram) {                             // entry 0: G in the arena; entry 1: X
        const void* As[2] = {plan->ws + plan->gram_off, A};
        void* Us[2] = {U, U};
        void* Ss[2] = {S, S};
        void* Vs[2] = {Vt, Vt};
        if (!A) return fail(HSVD_ERR_INVALID, "NULL data pointer");
        return execute_impl(*plan, As, Us, Ss, Vs, stream);
    }
    if (plan->mats.size() != 1) return fail(HSVD_ERR_INVALID, "batched plan: use hsvd_execute_batched");
    if (plan->rm_params) return learned_execute(*plan, A, U, S, Vt, stream);
    return execute_impl(*plan, &A, &U, &S, &Vt, stream);
}

hsvd_status hsvd_features_execute(hsvd_plan_t plan, const void* A, float* features, hipStream_t stream) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (plan->kind != 1) return fail(HSVD_ERR_INVALID, "not a feature plan");
    void* f = features;
    return execute_impl(*plan, &A, &f, &f, &f, stream);
}

hsvd_status hsvd_execute_batched(hsvd_plan_t plan, const void* const* A, void* const* U, void* const* S,
                                 void* const* Vt, hipStream_t stream) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (plan->kind != 0) return fail(HSVD_ERR_INVALID, "feature plan: use hsvd_features_execute");
    if (plan->gram) return fail(HSVD_ERR_INVALID, "Gram plan: use hsvd_execute");
    if (!A || !U || !S || !Vt) return fail(HSVD_ERR_INVALID, "NULL pointer array");
    return execute_impl(*plan, A, U, S, Vt, stream);
}

hsvd_status hsvd_set_profiling(hsvd_plan_t plan, int32_t enable) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (enable && !plan->seg_end.empty())
        return fail(HSVD_ERR_UNSUPPORTED, "per-launch timing is not recorded when Algorithm 2 stops on refine_eps");
    if (enable && plan->events.empty()) {
        plan->events.resize(plan->stages.size() + 2);
        for (auto& ev : plan->events) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    }
    plan->profiling = enable != 0;
    return HSVD_OK;
}

hsvd_status hsvd_launch_times(hsvd_plan_t plan, int32_t* kinds_host, float* ms_host, int32_t cap,
                              int32_t* count_host) {
    if (!plan || !count_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    const int n = (int)plan->stages.size() + 1;
    *count_host = n;
    if (!kinds_host || !ms_host) return HSVD_OK;
    if (!plan->profiling || plan->events.size() != (size_t)n + 1 || !plan->executed)
        return fail(HSVD_ERR_INVALID, "profiling was not enabled for the last execute");
    hipError_t e = hipEventSynchronize(plan->events.back());
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int i = 0; i < n && i < cap; ++i) {
        int kind = HSVD_LAUNCH_OUTPUT;
        if (i < (int)plan->stages.size()) {
            const Stage& s = plan->stages[i];
            switch (s.kind) {
                case ST_GEMM:
                    kind = s.bf16 ? (s.op == 0 ? HSVD_LAUNCH_GEMM_AX_BF16 : HSVD_LAUNCH_GEMM_ATX_BF16)
                         : s.f32  ? (s.op == 0 ? HSVD_LAUNCH_GEMM_AX_F32 : HSVD_LAUNCH_GEMM_ATX_F32)
                                  : (s.op == 0 ? HSVD_LAUNCH_GEMM_AX : HSVD_LAUNCH_GEMM_ATX);
                    break;
                case ST_TSQR_F: kind = HSVD_LAUNCH_TSQR_FACTOR; break;
                case ST_CQ1: case ST_CQ2: kind = HSVD_LAUNCH_CHOLQR; break;
                case ST_TSQR_A: kind = HSVD_LAUNCH_TSQR_APPLY; break;
                case ST_GRAM: kind = HSVD_LAUNCH_GRAM; break;
                case ST_REDUCE: kind = HSVD_LAUNCH_REDUCE; break;
                case ST_NN: kind = HSVD_LAUNCH_THIN_NN; break;
                case ST_SUM: kind = HSVD_LAUNCH_SUM; break;
                case ST_CORE: kind = s.maxdim > kCoreMaxN ? HSVD_LAUNCH_CORE_WIDE : HSVD_LAUNCH_CORE; break;
                case ST_ENERGY: case ST_ESUM: kind = HSVD_LAUNCH_ENERGY; break;
                case ST_FEAT: kind = HSVD_LAUNCH_FEATURES; break;
                case ST_LEAFCHECK: kind = HSVD_LAUNCH_CHECK; break;
                case ST_PQR: kind = HSVD_LAUNCH_PANEL_QR; break;
                case ST_GRAMX: kind = HSVD_LAUNCH_GRAM_XTX; break;
            }
        }
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, plan->events[i], plan->events[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        kinds_host[i] = kind;
        ms_host[i] = ms;
    }
    return HSVD_OK;
}

hsvd_status hsvd_launch_work(hsvd_plan_t plan, double* flops_host, double* bytes_host, int32_t cap,
                             int32_t* count_host) {
    if (!plan || !count_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    const hsvd_plan_st& P = *plan;
    const int n = (int)P.stages.size() + 1;
    *count_host = n;
    if (!flops_host || !bytes_host) return HSVD_OK;
    const unsigned char* b = P.blob.data();
    const double eA = P.opt.precision != HSVD_FP64 ? 4.0 : 8.0, e8 = 8.0;
    for (int i = 0; i < n && i < cap; ++i) {
        double f = 0.0, by = 0.0;
        if (i == n - 1) {                                   // output: U, Vt from the panels
            for (const MatDesc& M : P.mats)
                by += (double)(M.m + M.n) * M.pw * e8 + (double)(M.m + M.n) * M.k * eA + M.k * eA;
        } else {
            const Stage& s = P.stages[i];
            switch (s.kind) {
                case ST_GEMM: {
                    const GemmTask* T = (const GemmTask*)(b + s.tasks_off);
                    int ntask = 0;
                    const TileRef* R = (const TileRef*)(b + s.refs_off);
                    for (int t = 0; t < s.n; ++t) ntask = std::max(ntask, R[t].task + 1);
                    for (int t = 0; t < ntask; ++t) {
                        const double r = T[t].rows, c = T[t].cols, N = s.N;
                        f += 2.0 * r * c * N;
                        by += r * c * eA + (r + c) * N * e8;
                    }
                    break;
                }
                case ST_TSQR_F: {
                    const ChunkRef* C = (const ChunkRef*)(b + s.refs_off);
                    const TsqrTask* T = (const TsqrTask*)(b + s.tasks_off);
                    int ntask = 0;
                    for (int t = 0; t < s.n; ++t) ntask = std::max(ntask, C[t].task + 1);
                    for (int t = 0; t < ntask; ++t) {
                        if (T[t].cq_flag >= 0) continue;          // counted with the Cholesky passes
                        const double h = T[t].h, w = s.w, mn = std::min(h, w), mx = std::max(h, w);
                        f += 2.0 * mx * mn * mn - 2.0 * mn * mn * mn / 3.0;
                        by += 2.0 * h * w * e8;
                    }
                    break;
                }
                case ST_CQ1: case ST_CQ2: {                       // Gram of the panel + w^3 / 3
                    const ChunkRef* C = (const ChunkRef*)(b + s.refs_off);
                    const TsqrTask* T = (const TsqrTask*)(b + s.tasks_off);
                    int ntask = 0;
                    for (int t = 0; t < s.n; ++t) ntask = std::max(ntask, C[t].task + 1);
                    for (int t = 0; t < ntask; ++t) {
                        if (T[t].cq_flag < 0) continue;
                        const double h = T[t].h, w = s.w;
                        f += 2.0 * h * w * w + w * w * w;
                        by += (h * w + 2.0 * w * w) * e8;
                    }
                    break;
                }
                case ST_TSQR_A: {
                    const ChunkRef* C = (const ChunkRef*)(b + s.refs_off);
                    const TsqrTask* T = (const TsqrTask*)(b + s.tsqr_off);
                    const ApplyTask* A = (const ApplyTask*)(b + s.tasks_off);
                    int ntask = 0;
                    for (int t = 0; t < s.n; ++t) ntask = std::max(ntask, C[t].task + 1);
                    for (int t = 0; t < ntask; ++t) {
                        if (T[A[t].tsqr].cq_flag >= 0) continue;  // counted with the thin products
                        const double h = T[A[t].tsqr].h, w = s.w, c = s.c;
                        f += 4.0 * h * w * c;
                        by += (h * w + h * c) * e8;
                        if (A[t].add_u_off >= 0) {
                            f += 2.0 * h * A[t].add_w * c;
                            by += h * A[t].add_w * e8;
                        }
                    }
                    break;
                }
                case ST_GRAM: case ST_NN: case ST_REDUCE: case ST_SUM: {
                    const ThinTask* T = (const ThinTask*)(b + s.tasks_off);
                    int ntask = s.n;
                    if (s.kind != ST_REDUCE) {
                        const ChunkRef* C = (const ChunkRef*)(b + s.refs_off);
                        ntask = 0;
                        for (int t = 0; t < s.n; ++t) ntask = std::max(ntask, C[t].task + 1);
                    }
                    for (int t = 0; t < ntask; ++t) {
                        const ThinTask& x = T[t];
                        const double h = x.h, wx = x.wx, wy = x.wy;
                        if (s.kind == ST_GRAM) {
                            f += 2.0 * h * wx * wy;
                            by += h * (wx + wy) * e8;
                        } else if (s.kind == ST_NN) {
                            const double wx2 = x.x2_off >= 0 ? x.wx2 : 0.0;
                            f += 2.0 * h * (wx + wx2) * wy;
                            by += h * (wx + wx2 + 2.0 * wy) * e8;
                        } else if (s.kind == ST_REDUCE) {
                            const double nch = (x.h + P.thin_ch - 1) / P.thin_ch;
                            f += nch * wx * wy;
                            by += (nch + 1.0) * wx * wy * e8;
                        } else {                              // wx partial products of h x wy
                            f += (wx - 1.0) * h * wy;
                            by += (wx + 1.0) * h * wy * e8;
                        }
                    }
                    break;
                }
                case ST_CORE: {
                    const CoreTask* T = (const CoreTask*)(b + s.tasks_off);
                    for (int t = 0; t < s.n; ++t) {
                        const double d = (T[t].mode == CORE_MERGE) ? 2.0 * T[t].kcap : (double)T[t].dim;
                        f += 22.0 * d * d * d;
                        by += (d * d + d * T[t].out_w + T[t].out_w) * e8;
                    }
                    break;
                }
                case ST_ENERGY: {
                    const GemmTask* T = (const GemmTask*)(b + s.tasks_off);
                    for (int t = 0; t < s.n; ++t) {
                        f += 2.0 * T[t].rows * (double)T[t].cols;
                        by += (double)T[t].rows * T[t].cols * eA + e8;
                    }
                    break;
                }
                case ST_ESUM:                                     // partial sums of the fused pass
                    f = s.w;
                    by = (s.w + s.n) * e8;
                    break;
                case ST_LEAFCHECK:
                    f = 0.0;
                    by = 0.0;
                    break;
                case ST_GRAMX: {                                  // G = X^T X, symmetric: m n (n + 1) flops
                    const MatDesc& X = P.mats[1];
                    f = (double)X.m * X.n * (X.n + 1.0);
                    by = (double)X.m * X.n * eA + (double)X.n * X.n * e8;
                    break;
                }
                case ST_PQR: {                                    // a QR of the panel and its explicit Q
                    const TsqrTask* T = (const TsqrTask*)(b + s.tasks_off);
                    for (int t = 0; t < s.n; ++t) {
                        const double h = T[t].h, w = s.w, mn = std::min(h, w), mx = std::max(h, w);
                        f += 2.0 * (2.0 * mx * mn * mn - 2.0 * mn * mn * mn / 3.0);
                        by += 2.0 * h * w * e8;
                    }
                    break;
                }
                case ST_FEAT:
                    f = 40.0 * s.n;
                    by = s.n * (17.0 * e8 + 16.0 * 4.0);
                    break;
            }
        }
        flops_host[i] = f;
        bytes_host[i] = by;
    }
    return HSVD_OK;
}

hsvd_status hsvd_destroy(hsvd_plan_t plan) {
    if (!plan) return HSVD_OK;
    if (plan->executed) hipStreamSynchronize(plan->last_stream);
    for (auto& ev : plan->events) hipEventDestroy(ev);
    if (plan->gexec) hipGraphExecDestroy(plan->gexec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    if (plan->cap_stream) hipStreamDestroy(plan->cap_stream);
    for (hipStream_t bs : plan->bstreams) hipStreamDestroy(bs);
    for (hipEvent_t ev : plan->join_ev) hipEventDestroy(ev);
    if (plan->fork_ev) hipEventDestroy(plan->fork_ev);
    if (plan->rm_wplan) hsvd_destroy(plan->rm_wplan);
    if (plan->rm_features) hsvd_destroy(plan->rm_features);
    if (plan->rm_params) hipFree(plan->rm_params);
    if (plan->rm_feat) hipFree(plan->rm_feat);
    if (plan->rm_pred) hipFree(plan->rm_pred);
    if (plan->external) {             // device state in memory the plan does not own
        delete plan;
        return HSVD_OK;
    }
    if (plan->ws && !plan->ws_borrowed) hipFree(plan->ws);
    if (plan->iws && !plan->ws_borrowed) hipFree(plan->iws);
    if (plan->flags) hipFree(plan->flags);
    if (plan->dblob) hipFree(plan->dblob);
    if (plan->dptrs) hipFree(plan->dptrs);
    delete plan;
    return HSVD_OK;
}

hsvd_status hsvd_get_ranks(hsvd_plan_t plan, int32_t* r_host, int32_t count) {
    if (!plan || !r_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    if (count != (int32_t)plan->rank_slots.size()) return fail(HSVD_ERR_INVALID, "count does not match the plan");
    hipError_t e = hipSuccess;
    if (plan->executed) e = hipStreamSynchronize(plan->last_stream);
    std::vector<int> all((size_t)plan->iws_elems);
    if (e == hipSuccess && !all.empty())
        e = hipMemcpy(all.data(), plan->iws, sizeof(int) * all.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hsvd_get_ranks");
    for (int32_t i = 0; i < count; ++i) r_host[i] = all[(size_t)plan->rank_slots[i]];
    return HSVD_OK;
}

hsvd_status hsvd_get_leaf_info(hsvd_plan_t plan, int32_t* ranks, int32_t* fallback, int32_t count) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (plan->rm_ran && plan->rm_ran != plan) return hsvd_get_leaf_info(plan->rm_ran, ranks, fallback, count);
    if (plan->kind != 0 || count != (int32_t)plan->leaf_rank_slots.size())
        return fail(HSVD_ERR_INVALID, "count must be p * q of the plan's (first) matrix");
    hipError_t e = hipSuccess;
    if (plan->executed) e = hipStreamSynchronize(plan->last_stream);
    std::vector<int> all((size_t)plan->iws_elems);
    if (e == hipSuccess && !all.empty())
        e = hipMemcpy(all.data(), plan->iws, sizeof(int) * all.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hsvd_get_leaf_info");
    const MatDesc& M0 = plan->mats[0];
    for (int32_t b = 0; b < count; ++b) {
        // block b of the input's grid is logical block (j, i) of a transposed plan
        const int32_t lb = M0.trans ? (b % M0.p) * M0.q + b / M0.p : b;
        if (ranks) ranks[b] = all[(size_t)plan->leaf_rank_slots[lb]];
        if (fallback) fallback[b] = plan->leaf_flag_slots[lb] >= 0 ? all[(size_t)plan->leaf_flag_slots[lb]] : 0;
    }
    return HSVD_OK;
}

hsvd_status hsvd_get_refine_iterations(hsvd_plan_t plan, int32_t* iters_host) {
    if (!plan || !iters_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    if (plan->kind != 0) return fail(HSVD_ERR_INVALID, "feature plan");
    *iters_host = plan->refine_done;
    return HSVD_OK;
}

hsvd_status hsvd_get_rank(hsvd_plan_t plan, int32_t* r_host) {
    if (!plan || !r_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    if (plan->rm_ran && plan->rm_ran != plan) return hsvd_get_rank(plan->rm_ran, r_host);
    if (plan->rank_slots.size() != 1) return fail(HSVD_ERR_INVALID, "batched plan: use hsvd_get_ranks");
    return hsvd_get_ranks(plan, r_host, 1);
}

hsvd_status hsvd_get_status(hsvd_plan_t plan, uint32_t* flags_host) {
    if (!plan || !flags_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    if (plan->rm_ran && plan->rm_ran != plan) {
        hsvd_status st = hsvd_get_status(plan->rm_ran, flags_host);
        if (st == HSVD_OK && plan->rm_refits > 0) *flags_host |= HSVD_FLAG_RANK_FALLBACK;
        return st;
    }
    hipError_t e = hipSuccess;
    if (plan->executed) e = hipStreamSynchronize(plan->last_stream);
    unsigned fl[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(fl, plan->flags, 2 * sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hsvd_get_status");
    *flags_host = (fl[0] & 0xFFFFu) | (std::min(fl[1], 0xFFFFu) << 16);
    return HSVD_OK;
}

hsvd_status hsvd_get_tuning(hsvd_plan_t plan, int32_t* thin_rows, int32_t* merge_qr, int32_t* leaf_qr,
                            int32_t* tuned, float* tuned_ms) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (thin_rows) *thin_rows = plan->thin_ch;
    if (merge_qr) *merge_qr = plan->merge_qr;
    if (leaf_qr) *leaf_qr = plan->leaf_qr;
    if (tuned) *tuned = plan->tuned;
    if (tuned_ms) *tuned_ms = plan->tuned_ms;
    return HSVD_OK;
}

hsvd_status hsvd_workspace_bytes(hsvd_plan_t plan, size_t* bytes_host) {
    if (!plan || !bytes_host) return fail(HSVD_ERR_INVALID, "NULL argument");
    *bytes_host = workspace_need(*plan);
    return HSVD_OK;
}

hsvd_status hsvd_set_rank_model(hsvd_plan_t plan, const void* weights_host, size_t bytes) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (plan->kind != 0 || plan->mats.size() != 1 || plan->external || !plan->leaf_width.empty() || plan->trans)
        return fail(HSVD_ERR_INVALID, "rank models attach to single-matrix plans from hsvd_plan / hsvd_plan_ex "
                                      "that merge row slabs last");
    if (plan->opt.precision != HSVD_FP64 && plan->opt.precision != HSVD_FP32)
        return fail(HSVD_ERR_UNSUPPORTED, "rank models need a float64 or float32-storage plan");
    if (weights_host && bytes != sizeof(float) * (size_t)kMlpParams)
        return fail(HSVD_ERR_INVALID, "weights must be HSVD_RANK_MODEL_PARAMS floats");
    hipError_t e = hipSuccess;
    if (plan->executed) e = hipStreamSynchronize(plan->last_stream);
    if (e != hipSuccess) return hip_fail(e, "hsvd_set_rank_model");
    if (!weights_host) {                              // detach
        if (plan->rm_wplan) hsvd_destroy(plan->rm_wplan);
        if (plan->rm_features) hsvd_destroy(plan->rm_features);
        if (plan->rm_params) hipFree(plan->rm_params);
        if (plan->rm_feat) hipFree(plan->rm_feat);
        if (plan->rm_pred) hipFree(plan->rm_pred);
        plan->rm_wplan = plan->rm_features = plan->rm_ran = nullptr;
        plan->rm_params = plan->rm_feat = plan->rm_pred = nullptr;
        plan->rm_widths.clear();
        return HSVD_OK;
    }
    const MatDesc& M = plan->mats[0];
    const int nb = M.p * M.q;
    if (!plan->rm_params) {
        e = hipMalloc(&plan->rm_params, sizeof(float) * kMlpParams);
        if (e == hipSuccess) e = hipMalloc(&plan->rm_feat, sizeof(float) * 16 * (size_t)nb);
        if (e == hipSuccess) e = hipMalloc(&plan->rm_pred, sizeof(float) * (size_t)nb);
        if (e != hipSuccess) return fail(HSVD_ERR_ALLOC, "rank model allocation failed");
        hsvd_options fo;
        hsvd_default_options(&fo);
        fo.precision = plan->opt.precision;
        fo.seed = plan->opt.seed;
        fo.graph = plan->opt.graph;
        int64_t m = M.m, n = M.n;
        int32_t p = M.p, q = M.q, one = 1;
        hsvd_status st = plan_impl(&plan->rm_features, 1, &m, &n, &p, &q, &one, 0.0, &fo, nullptr, nullptr, 1, false);
        if (st != HSVD_OK) return st;
    }
    e = hipMemcpy(plan->rm_params, weights_host, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hsvd_set_rank_model");
    plan->rm_ran = nullptr;
    return HSVD_OK;
}

hsvd_status hsvd_get_leaf_widths(hsvd_plan_t plan, int32_t* widths_host, int32_t count, int32_t* refits_host,
                                 int32_t* plain_host) {
    if (!plan) return fail(HSVD_ERR_INVALID, "plan is NULL");
    if (!plan->rm_params) return fail(HSVD_ERR_INVALID, "no rank model attached");
    if (widths_host && count != (int32_t)plan->rm_widths.size())
        return fail(HSVD_ERR_INVALID, "count must be p * q (after a learned execute)");
    if (widths_host)
        for (int32_t b = 0; b < count; ++b) widths_host[b] = plan->rm_widths[(size_t)b];
    if (refits_host) *refits_host = plan->rm_refits;
    if (plain_host) *plain_host = plan->rm_plain;
    return HSVD_OK;
}

hsvd_status hsvd_set_workspace(hsvd_plan_t plan, void* dptr, size_t bytes) {
    if (!plan || !dptr) return fail(HSVD_ERR_INVALID, "NULL argument");
    if (plan->external) return fail(HSVD_ERR_INVALID, "not a plan from hsvd_plan*");
    if ((uintptr_t)dptr % 256) return fail(HSVD_ERR_INVALID, "workspace must be 256-byte aligned");
    const size_t need = workspace_need(*plan);
    if (bytes < need)
        return fail(HSVD_ERR_INVALID, "workspace of " + std::to_string(bytes) + " bytes; the plan needs " +
                                          std::to_string(need));
    hipError_t e = hipSuccess;
    if (plan->executed) e = hipStreamSynchronize(plan->last_stream);
    const size_t ws_bytes = sizeof(double) * (size_t)std::max<int64_t>(plan->ws_elems, 32);
    const size_t iw_off = (ws_bytes + 255) / 256 * 256;
    unsigned char* b = (unsigned char*)dptr;
    if (e == hipSuccess && (unsigned char*)plan->ws != b)
        e = hipMemcpy(b, plan->ws, ws_bytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess && (unsigned char*)plan->iws != b + iw_off)
        e = hipMemcpy(b + iw_off, plan->iws, sizeof(int) * (size_t)std::max(plan->iws_elems, 1),
                      hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();       // copies done before the old memory goes
    if (e != hipSuccess) return hip_fail(e, "hsvd_set_workspace");
    if (!plan->ws_borrowed) {
        hipFree(plan->ws);
        hipFree(plan->iws);
    }
    plan->ws = (double*)b;
    plan->iws = (int*)(b + iw_off);
    plan->ws_borrowed = true;
    // a captured graph holds the old addresses: the next execute captures again
    if (plan->gexec) hipGraphExecDestroy(plan->gexec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    plan->gexec = nullptr;
    plan->graph = nullptr;
    return HSVD_OK;
}

const char* hsvd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------ allocation-free entry point
// The whole device state of one call (arena, int arena, status flags, task tables and the
// pointer table) placed in a file-scope device array instead of hipMalloc'd memory.  In
// host code `scratch` names a host-side stand-in: its device address is taken once per
// device with hipGetSymbolAddress and only that address is used.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;   // per device: the address of that device's copy

hsvd_status static_scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e,
                                                   "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return HSVD_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

extern "C" {

hsvd_status hsvd_svd_static(int64_t m, int64_t n, int32_t p, int32_t q, int32_t k, double tol,
                            const hsvd_options* opt, const void* A, void* U, void* S, void* Vt,
                            int32_t* r_host, hipStream_t stream) {
    if (!A || !U || !S || !Vt) return fail(HSVD_ERR_INVALID, "NULL data pointer");
    hsvd_plan_t P = nullptr;
    hsvd_status st = plan_impl(&P, 1, &m, &n, &p, &q, &k, tol, opt, nullptr, nullptr, 0, true);
    if (st != HSVD_OK) return st;
    std::unique_ptr<hsvd_plan_st> hold(P);
    P->external = true;
    // layout: arena | int arena | flags | task blob | pointer table, 256-byte aligned
    const size_t off_iws = align256(sizeof(double) * (size_t)std::max<int64_t>(P->ws_elems, 32));
    const size_t off_flags = align256(off_iws + sizeof(int) * (size_t)std::max(P->iws_elems, 1));
    const size_t off_blob = align256(off_flags + sizeof(unsigned) * 4);
    const size_t off_ptrs = align256(off_blob + std::max<size_t>(P->blob.size(), 256));
    const size_t total = align256(off_ptrs + sizeof(void*) * 4);
    if (total > kStaticScratchBytes)
        return fail(HSVD_ERR_INVALID, "hsvd_svd_static: this problem needs " + std::to_string(total) +
                                          " bytes of device state; the allocation-free entry point holds at most " +
                                          std::to_string(kStaticScratchBytes));
    void* base = nullptr;
    st = static_scratch_address(&base);
    if (st != HSVD_OK) return st;
    if (hipError_t pe = prepare_launches(); pe != hipSuccess) return hip_fail(pe, "kernel attributes");
    unsigned char* b = (unsigned char*)base;
    P->ws = (double*)b;
    P->iws = (int*)(b + off_iws);
    P->flags = (unsigned*)(b + off_flags);
    P->dblob = b + off_blob;
    P->dptrs = (void**)(b + off_ptrs);
    // the array keeps the previous call's contents: clear all of it (a kernel, no memset),
    // then the task tables, the constant panels and the Gaussian test matrices
    hipError_t e = launch_fill(P->ws, (int64_t)(total / sizeof(double)), 0.0, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P->dblob, P->blob.data(), P->blob.size(), hipMemcpyHostToDevice, stream);
    for (auto& c : P->ws_init)
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->ws + c.first, c.second.data(), c.second.size() * sizeof(double),
                               hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_gaussian(P->ws + P->omega_off, P->omega_count, P->opt.seed, stream);
    if (e != hipSuccess) return hip_fail(e, "hsvd_svd_static: set-up");
    st = execute_impl(*P, &A, &U, &S, &Vt, stream);
    if (st != HSVD_OK) {
        hipStreamSynchronize(stream);
        return st;
    }
    int32_t r = 0;
    e = hipMemcpyAsync(&r, P->iws + P->rank_slots[0], sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hsvd_svd_static");
    if (r_host) *r_host = r;
    return HSVD_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ learned rank model
struct hsvd_rank_model_st {
    float* params = nullptr;   // float32 masters (the network uses them rounded to float16)
    float* m1 = nullptr;       // Adam moments
    float* m2 = nullptr;
    int steps_done = 0;        // Adam step counter
    int batches_done = 0;      // minibatch counter (which samples the next step takes)
};

extern "C" {

hsvd_status hsvd_rank_model_create(hsvd_rank_model_t* out, uint64_t seed) {
    if (!out) return fail(HSVD_ERR_INVALID, "out is NULL");
    *out = nullptr;
    hsvd_rank_model_st* M = new (std::nothrow) hsvd_rank_model_st();
    if (!M) return fail(HSVD_ERR_ALLOC, "host allocation failed");
    hipError_t e = hipMalloc(&M->params, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&M->m1, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&M->m2, sizeof(float) * kMlpParams);
    if (e != hipSuccess) { hsvd_rank_model_destroy(M); return fail(HSVD_ERR_ALLOC, "allocation failed"); }
    // He initialisation: W1 ~ N(0, 2/16), W2 ~ N(0, 2/64), w3 ~ N(0, 1/64), biases 0,
    // output bias 3 (log2 of a middling rank)
    std::vector<float> h(kMlpParams, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < 64 * 16; ++i) h[i] = (float)(nd(rng) * std::sqrt(2.0 / 16.0));
    for (int i = 0; i < 64 * 64; ++i) h[1088 + i] = (float)(nd(rng) * std::sqrt(2.0 / 64.0));
    for (int i = 0; i < 64; ++i) h[5248 + i] = (float)(nd(rng) * std::sqrt(1.0 / 64.0));
    h[kMlpParams - 1] = 3.0f;
    e = hipMemcpy(M->params, h.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(M->m1, 0, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMemset(M->m2, 0, sizeof(float) * kMlpParams);
    if (e != hipSuccess) { hsvd_rank_model_destroy(M); return hip_fail(e, "rank model init"); }
    *out = M;
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_destroy(hsvd_rank_model_t model) {
    if (!model) return HSVD_OK;
    hipDeviceSynchronize();
    if (model->params) hipFree(model->params);
    if (model->m1) hipFree(model->m1);
    if (model->m2) hipFree(model->m2);
    delete model;
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_set_params(hsvd_rank_model_t model, const float* params_host, int32_t count) {
    if (!model || !params_host || count != kMlpParams) return fail(HSVD_ERR_INVALID, "bad argument");
    hipError_t e = hipMemcpy(model->params, params_host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(model->m1, 0, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMemset(model->m2, 0, sizeof(float) * kMlpParams);
    if (e != hipSuccess) return hip_fail(e, "hsvd_rank_model_set_params");
    model->steps_done = model->batches_done = 0;
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_get_params(hsvd_rank_model_t model, float* params_host, int32_t count) {
    if (!model || !params_host || count != kMlpParams) return fail(HSVD_ERR_INVALID, "bad argument");
    hipError_t e = hipMemcpy(params_host, model->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hsvd_rank_model_get_params");
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_train(hsvd_rank_model_t model, const float* X, const float* T, int32_t count,
                                  int32_t steps, float lr, float* losses, hipStream_t stream) {
    if (!model || !X || !T || count < 1 || steps < 1 || !(lr > 0.0f))
        return fail(HSVD_ERR_INVALID, "bad argument");
    hipError_t e = launch_mlp_train(model->params, model->m1, model->m2, X, T, count, steps,
                                    model->batches_done, model->steps_done, lr, nullptr, losses, stream);
    if (e != hipSuccess) return hip_fail(e, "rank model training launch");
    model->steps_done += steps;
    model->batches_done += steps;
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_grad(hsvd_rank_model_t model, const float* X, const float* T, int32_t count,
                                 int32_t batch_index, float* grad, float* loss, hipStream_t stream) {
    if (!model || !X || !T || !grad || !loss || count < 1 || batch_index < 0)
        return fail(HSVD_ERR_INVALID, "bad argument");
    hipError_t e = launch_mlp_train(model->params, model->m1, model->m2, X, T, count, 0, batch_index, 0,
                                    0.0f, grad, loss, stream);
    if (e != hipSuccess) return hip_fail(e, "rank model gradient launch");
    return HSVD_OK;
}

hsvd_status hsvd_rank_model_predict(hsvd_rank_model_t model, const float* X, int32_t count, float* out,
                                    hipStream_t stream) {
    if (!model || !X || !out || count < 0) return fail(HSVD_ERR_INVALID, "bad argument");
    hipError_t e = launch_mlp_predict(model->params, X, count, out, stream);
    if (e != hipSuccess) return hip_fail(e, "rank model prediction launch");
    return HSVD_OK;
}

}  // extern "C"
