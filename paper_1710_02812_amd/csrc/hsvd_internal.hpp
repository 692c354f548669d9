// Internal task descriptors shared by the host plan and the gfx950 kernels.
//
// Every device buffer lives in one plan-owned arena of doubles (offsets are in
// elements of that arena) plus a small int arena (ranks, tree counters, flags).
// The input A is addressed by element offsets from the pointer passed to execute.
// Panels are column-major with an explicit leading dimension; A is row-major.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsvd {

constexpr double kEps = 2.220446049250313e-16;   // 2^-52

// ---------------------------------------------------------------- big products with A
// op 0: Y (rows x N) = A_blk (rows x cols) * X (cols x N)
// op 1: Y (cols x N) = A_blk^T * X (rows x N)
struct GemmTask {
    int64_t a_off;        // offset of A_blk[0][0] in its matrix (row-major, leading dim lda)
    int64_t x_off, y_off; // arena offsets (col-major panels)
    int64_t lda;          // leading dimension (columns) of the task's matrix
    int32_t rows, cols;   // A_blk shape as stored
    int32_t x_ld, y_ld;
    int32_t tiles;        // output row tiles of this task
    int32_t mat;          // matrix index: A = Aptrs[mat]
};
struct TileRef { int32_t task; int32_t tile; };
// Column tiles of a float64 matrix-core pass over N output columns: one 64 x 96 tile up to
// 96 columns (A read once), else 64-column tiles.
__host__ __device__ inline int gemm_f64_col_tiles(int N) { return (N > 64 && N <= 96) ? 1 : (N + 63) / 64; }
// A block's energy from the partial sums of the tiles that read it (a fused sketch pass).
struct EnergySum { int64_t out; int32_t first, count; };
// A tile of the Gram matrix G = X^T X (upper triangle, ti <= tj) over one row chunk of X.
struct GramRef { int32_t ti, tj, chunk, pad; };

// ---------------------------------------------------------------- tall-skinny QR (TSQR)
// Panel P (h x w, col-major, ld) split into nch row chunks of `ch` rows; each chunk
// gets a Householder QR in LDS, then R factors are merged pairwise up a binary tree
// (the last work-group to finish a pair merges it).  Tree node (level L, index i)
// has children (2i, 2i+1) at level L-1; an odd last node passes straight up.
struct TsqrTask {
    int64_t p_off;        // panel, overwritten by the chunk reflectors
    int64_t store_off;    // per-node storage: R (w*w) | V (F w * w) | tau (w) | T (w*w)
    int64_t r_out;        // final R (w x w, col-major, ld w), upper triangular
    int32_t h, p_ld;
    int32_t nch;          // chunks
    int32_t chunk0;       // first flat chunk index of this task
    int32_t cnt_off;      // int arena: one counter per tree node
    int32_t levels;       // tree levels above the chunks
    // Cholesky QR fast path (cq_flag < 0: none): scratch (cq_size doubles), the int
    // slot of its outcome (0: the Cholesky outputs stand, 1: the Householder kernels
    // run) and the first of its cq_nodes arrival counters (one when nch = 1)
    int64_t cq_off = 0;
    int32_t cq_flag = -1, cq_cnt = -1;
    // one-launch panel QR (k_panel_qr; pq_q_off < 0: none): explicit Q written to
    // pq_q_off (h x w, ld pq_q_ld, not overlapping the panel), R to r_out when asked,
    // 2 w^2 doubles of scratch at pq_scr; its outcome goes to cq_flag as above
    int64_t pq_q_off = -1, pq_scr = 0;
    int32_t pq_q_ld = 0, pq_pad = 0;
};
struct ChunkRef { int32_t task; int32_t chunk; };

constexpr int THIN_CH = 128;    // rows per chunk of the thin-panel products

constexpr int kTsqrMaxW = 80;
// Fan-in F of the R-factor tree: up to F stacked w x w factors are merged by one
// Householder QR held in registers (4w <= 256 rows for w <= 64, 2w <= 160 above).
__host__ __device__ inline int tsqr_fanin(int w) { return w <= 64 ? 4 : 2; }
// Tree nodes (chunks included) and levels above the chunks for nch chunks.
__host__ __device__ inline int tsqr_nodes(int nch, int F) {
    int nodes = 0;
    for (int n = nch;; n = (n + F - 1) / F) {
        nodes += n;
        if (n == 1) break;
    }
    return nodes;
}
__host__ __device__ inline int tsqr_levels(int nch, int F) {
    int l = 0;
    for (int n = nch; n > 1; n = (n + F - 1) / F) ++l;
    return l;
}
// Per-node storage: R (w*w) | V (F w * w, ld F w) | tau (w) | T (w*w).
__host__ __device__ inline int64_t tsqr_slot_size(int w) { return (int64_t)(tsqr_fanin(w) + 2) * w * w + w; }
// Rows per chunk: the factor kernel holds a chunk in registers: 16 lanes x 16 rows
// per column (w <= 64) or 16 lanes x 10 rows (w <= 80).
inline int tsqr_chunk_rows(int w) { return w <= 64 ? 256 : 160; }

// out (h x c) = Q * X  (+ U1 * T when add_u_off >= 0), Q the explicit thin factor of a
// TsqrTask, X (w x c).  One work-group per chunk.
struct ApplyTask {
    int32_t tsqr;         // index into the TsqrTask array of the same launch family
    int32_t out_ld;
    int64_t x_off;        // X, col-major, ld w
    int64_t out_off;
    int64_t add_u_off;    // U1 panel (h x w1, ld add_u_ld) or -1
    int64_t add_t_off;    // T (w1 x c, col-major, ld w1)
    int32_t add_u_ld, add_w;
};

// ---------------------------------------------------------------- thin panel algebra
// Row-chunked ops on col-major panels of height h:
//   gram:  part[c] = X_c^T Y_c           (wx x wy), per chunk c
//   reduce:C = sum_c part[c]; Cacc (+)= C  (one group per task)
//   sub:   Y_c -= X_c * C
//   nn:    O_c (+)= X_c * T (+ X2_c * T2)
struct ThinTask {
    int64_t x_off, y_off, c_off, part_off, acc_off;
    int32_t h, x_ld, y_ld, c_ld;
    int32_t wx, wy;       // widths
    int32_t nch, chunk0;
    int32_t accumulate;   // reduce: 0 -> Cacc = C, 1 -> Cacc += C; nn: 0 set, 1 add, 2 sub
    int32_t cond = -1;    // nn: runs only while iws[cond] == 0 (a Cholesky QR outcome), or always
    // nn: a second product X2_c * C2 (X2 h x wx2, ld x2_ld; C2 wx2 x wy, ld c2_ld) summed
    // with the first before the store (x2_off < 0: none)
    int64_t x2_off = -1, c2_off = 0;
    int32_t x2_ld = 0, c2_ld = 0, wx2 = 0, pad2 = 0;
};

// ---------------------------------------------------------------- Jacobi cores
enum CoreMode : int32_t {
    CORE_UPPER = 0,       // M = R (dim x dim) read from m_off (ld m_ld)
    CORE_UPPER_T = 1,     // M = R^T
    CORE_MERGE = 2,       // M = E = [[S1, C S2], [0, R S2]] (compact r1 + r2)
    CORE_DENSE = 3        // M = a dense dim x dim matrix (kernel-level tests)
};
struct CoreTask {
    int32_t mode;
    int32_t dim;          // UPPER modes: dimension of R as stored (panel width)
    int64_t m_off; int32_t m_ld;
    int32_t rank_in;      // UPPER modes: int-arena slot holding the active size, or -1 (= dim)
    // merge inputs
    int64_t s1_off, s2_off, c_off, r_off;
    int32_t c_ld, r_ld;
    int32_t rank1, rank2; // int-arena slots
    // outputs
    int64_t u_off; int32_t u_ld;   // left vectors: UPPER -> rows 0..dim-1; MERGE -> rows r1..r1+r2-1
    int64_t t_off; int32_t t_ld;   // MERGE: left-vector rows 0..r1-1
    int64_t v_off; int32_t v_ld;   // accumulated right rotations (or -1)
    int64_t sig_off;               // kcap values, zero padded
    int32_t out_w;                 // columns written to u/t/v outputs (zero padded past r)
    int32_t rank_out;              // int-arena slot for r
    int32_t kcap, rule;
    double tol;
    int32_t floor_rows;            // zero-floor shape: max(floor_rows, floor_cols or r1+r2)
    int32_t floor_cols;            // < 0: use the active core size
    int32_t fixed_rank_slot;       // >= 0: rank = min(zero-floor count, ranks[slot])
    int32_t precond;               // 1: LQ-precondition (left vectors only; needs v_off < 0)
    // a-posteriori check of a leaf whose block energy E is known (energy_off >= 0):
    // iws[flag_slot] = 1 (and status bit 4) when E - sum(sigma^2) > tol^2 E
    int64_t energy_off;
    int32_t flag_slot;
    int32_t pad2;
    // >= 0: all singular values of the core (sorted, zero past its size), dim of them,
    // before truncation (the leaves' power-step convergence test reads them)
    int64_t sigall_off = -1;
    // > 0: the sweeps stop once no pair has |g_a . g_b| > orth_tol |g_a| |g_b|; else the
    // working-precision threshold max(rows, 1) 2^-52
    double orth_tol = 0.0;
    // cores of more than kCoreMaxN columns: a kWideScratch-element float64 scratch panel
    // that holds the core's columns while it is decomposed (else -1)
    int64_t scr_off = -1;
};

// Core sizes: LDS-resident cores up to kCoreMaxN columns (accumulated right vectors up
// to kCoreMaxV); merge and dense cores up to kWideCoreMaxN columns keep their columns in
// a scratch panel of kWideCoreRows x kWideCoreMaxN.
constexpr int kCoreMaxN = 128;
constexpr int kCoreMaxV = 96;
constexpr int kWideCoreMaxN = 160;
constexpr int kWideCoreRows = 160;
constexpr int64_t kWideScratch = (int64_t)kWideCoreRows * kWideCoreMaxN;
// Rank cap of a plan: merge cores of 2k columns must fit the wide cores.
constexpr int kMaxRank = kWideCoreMaxN / 2;

// Column-orthogonality threshold of the mixed-precision plans' tree cores (leaves,
// merges, slab re-projections): their inputs carry bfloat16 rounding (2^-9, about 2e-3
// relative), so cosines of 1e-5, two orders below it, leave left vectors whose error
// (about the threshold times sigma_1 over the gap at the cut) stays below the input's
// own; the projection and Algorithm 2 cores, which set the output's orthonormality and
// refine against the unrounded input, keep the working-precision threshold.
constexpr double kMixedOrthTol = 1e-5;
// The same for float32-storage plans, whose inputs carry float32 rounding (2^-24,
// about 6e-8): 1e-9, two orders below it.
constexpr double kF32OrthTol = 1e-9;

// ---------------------------------------------------------------- output
struct OutputArgs {
    int64_t u_off, v_off, sig_off;  // final U (m x W), V (n x W) panels, sigma
    int32_t u_ld, v_ld;
    int32_t m, n, k;
    int32_t rank_slot;
    int32_t sign_off;               // int arena: k signs
    int32_t pad;
};
// Stopping test of Algorithm 2 for one matrix: singular values of two consecutive
// iterations (sig_old, sig_new, each rank_slot entries) compared in the 2-norm.
struct RefineCheck {
    int64_t sig_old, sig_new;
    int32_t rank_slot, pad;
};
// Per-execute pointer table of a plan over `count` matrices: entries
// [4 i .. 4 i + 3] are A, U, S, Vt of matrix i (device pointers).

// ---------------------------------------------------------------- learned block rank
constexpr int kMlpParams = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1;   // 5313
constexpr int kMlpBatch = 64;

// Device state of the allocation-free entry point (a file-scope device array).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;

// ---------------------------------------------------------------- launches
// Raises a kernel's dynamic-LDS limit once per device (bit dev of *done); plans call
// prepare_launches() at creation so that no attribute is set during a graph capture.
inline hipError_t set_lds_limit_once(const void* fn, int bytes, unsigned long long* done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned long long bit = 1ull << (dev & 63);
    if (__atomic_load_n(done, __ATOMIC_ACQUIRE) & bit) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) __atomic_fetch_or(done, bit, __ATOMIC_RELEASE);
    return e;
}
hipError_t prepare_core_launches();
hipError_t prepare_core_wide();
hipError_t prepare_panel_qr_launches();
hipError_t prepare_gemm_bf16_launches();
hipError_t prepare_gemm_f32_launches();

// All launchers enqueue on `s` and return the hipError_t of the launch.
// `guard` (device int or nullptr): when it points at a non-zero value every work-group
// of the launch returns at once (stages of an iteration that has already stopped).
// bfloat16 matrix-core passes: strips of 256 output rows holding all N <= 96 output
// columns (TileRef.tile = strip index), so that each element of A is read once
constexpr int kBf16TileRows = 256;
constexpr int kBf16MaxN = 96;
hipError_t launch_gemm_bf16(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                            const TileRef* tiles, int ntiles, int N, hipStream_t s);
// float32 matrix-core passes (mixed plans' float32-accurate products): same strips
hipError_t launch_gemm_f32(int op, const void* const* ptrs, double* ws, const GemmTask* tasks,
                           const TileRef* tiles, int ntiles, int N, hipStream_t s);
// G = X^T X partials: one per row chunk of `rows_per_chunk` rows of matrix `mat`
// (X row-major m x n, float32 or float64); partial c at ws + parts_off + c n^2.
hipError_t launch_gram_xtx(int fp32, const void* const* ptrs, int mat, int64_t m, int64_t n,
                           int64_t rows_per_chunk, double* ws, int64_t parts_off, const GramRef* refs, int nrefs,
                           hipStream_t s);
// e_part >= 0 (op 0 only): tile i also writes its part of its block's energy (the
// squares of the A rows it reads; 0 from column tiles past the first) to ws[e_part + i].
hipError_t launch_gemm(int op, int fp32, const void* const* ptrs, double* ws,
                       const GemmTask* tasks, const TileRef* tiles, int ntiles, int N,
                       hipStream_t s, const int* guard = nullptr, int64_t e_part = -1);
hipError_t launch_tsqr_factor(double* ws, int* iws, const TsqrTask* tasks,
                              const ChunkRef* chunks, int nchunks, int w, int ch,
                              hipStream_t s, const int* guard = nullptr);
// Panel QR of the leaves (one work-group per TsqrTask with pq_q_off >= 0, w <= kPanelQrMaxW):
// repeated Cholesky QR, the first pass shifted; need_r 1 also forms R at r_out, and
// kPqrSpanOnly stops after the shifted first pass (Q spans the panel and is well
// conditioned but not orthonormal to working precision; no R), for a sketch whose Q only
// feeds the next power step.
constexpr int kPqrSpanOnly = 2;          // panel QR mode: the shifted first pass only
constexpr int kPanelQrMaxW = 96;
constexpr int kPanelQrMaxPass = 4;
// `order` (device, ntasks task indices, or nullptr for task order): the dispatch order
hipError_t launch_panel_qr(double* ws, int* iws, const TsqrTask* tasks, int ntasks, int w, int need_r,
                           hipStream_t s, const int* guard = nullptr, const int* order = nullptr);
hipError_t launch_tsqr_apply(double* ws, const int* iws, const TsqrTask* tsqr, const ApplyTask* tasks,
                             const ChunkRef* chunks, int nchunks, int w, int ch, int c,
                             hipStream_t s, const int* guard = nullptr);
// tx, ty: 64-column tiles of the widest X and Y of the tasks (1 or 2)
hipError_t launch_thin_gram(double* ws, const ThinTask* t, const ChunkRef* chunks,
                            int nchunks, int chh, hipStream_t s, int tx = 2, int ty = 2);
// maxsz: the largest wx * wy over the tasks (grid: task x element slices of 256)
hipError_t launch_thin_reduce(double* ws, const ThinTask* t, int ntasks, int maxsz, hipStream_t s);
hipError_t launch_thin_nn(double* ws, const int* iws, const ThinTask* t, const ChunkRef* chunks,
                          int nchunks, int chh, hipStream_t s, int ty = 2);
// Cholesky QR pass 1 or 2 over the chunks of TsqrTasks with cq_flag >= 0 (w <= 64)
hipError_t launch_cholqr(int pass, double* ws, int* iws, const TsqrTask* tasks, const ChunkRef* chunks,
                         int nchunks, int w, int ch, hipStream_t s);
// The chunks' partial Grams are summed up a tree of fan-in kCqFan: cq_nodes counts its
// nodes above the chunks (one arrival counter each; each holds a stored w x w sum).
constexpr int kCqFan = 8;
__host__ __device__ inline int cq_up(int n) { return (n + kCqFan - 1) / kCqFan; }
__host__ __device__ inline int cq_nodes(int nch) {
    int s = 0;
    for (int n = nch; n > 1; n = cq_up(n)) s += cq_up(n);
    return s;
}
// Scratch of a panel: R1 | M1 | M2 | chunk parts (nch w^2) | node sums | Q1 (h x w, ld h)
__host__ __device__ inline int64_t cq_q1(int w, int nch) { return (int64_t)(3 + nch + cq_nodes(nch)) * w * w; }
__host__ __device__ inline int64_t cq_size(int w, int nch, int h) { return cq_q1(w, nch) + (int64_t)h * w; }
hipError_t launch_thin_sum(double* ws, const ThinTask* t, const ChunkRef* chunks,
                           int nchunks, int chh, hipStream_t s);
hipError_t launch_core(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                       int max_sweeps, unsigned* flags, int with_v, hipStream_t s,
                       const int* guard = nullptr);
hipError_t launch_core_wide(double* ws, int* iws, const CoreTask* tasks, int ntasks, int maxdim,
                            int max_sweeps, unsigned* flags, hipStream_t s, const int* guard);
// Peak probes (measurement only): kind 0 read, 1 copy, 2 / 3 / 4 float64 / bfloat16 /
// float32 matrix cores; `sink` holds 2048 floats; *work gets the bytes or flops.
hipError_t launch_probe(int kind, void* buf, int64_t bytes, int iters, float* sink, double* work,
                        hipStream_t s);
hipError_t launch_mlp_train(float* master, float* m1, float* m2, const float* X, const float* T,
                            int count, int steps, int s0, int t0, float lr, float* grad_out,
                            float* loss_out, hipStream_t s);
hipError_t launch_mlp_predict(const float* master, const float* X, int count, float* out, hipStream_t s);
hipError_t launch_block_energy(const void* const* ptrs, int fp32, const GemmTask* tasks, int ntasks,
                               double* ws, int64_t out_off, hipStream_t s);
// ws[t.out] = sum of ws[part_off + t.first + c], c < t.count, in that order, per task.
hipError_t launch_energy_sum(double* ws, int64_t part_off, const EnergySum* tasks, int ntasks, hipStream_t s);
hipError_t launch_block_features(const double* ws, int64_t sig_off, int64_t energy_off, int nblocks,
                                 float* out, hipStream_t s);
hipError_t launch_gaussian(double* out, int64_t count, uint64_t seed, hipStream_t s);
hipError_t launch_gaussian_f32(float* out, int64_t count, uint64_t seed, hipStream_t s);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
// iws[out_slot] = 1 when every item has ||s_new - s_old||^2 <= eps^2 ||s_old||^2 over
// its rank, else 0 (one work-group).
hipError_t launch_refine_check(const double* ws, int* iws, const RefineCheck* items, int count, double eps,
                               int out_slot, hipStream_t s);
// Convergence test of the leaves' power steps (one item per leaf): after step t the
// leaf's core has given the sketch's singular values s_0 >= ... >= s_{w-1} (zero past
// its numerical rank); with r the leaf's truncation rank, the leaf has converged when
// r == 0, s_{w-1} == 0, or (s_{w-1} / s_{r-1})^(2t+1) <= kLeafConvTol.  The subspace
// iteration bound carries a factor set by the test matrix (the conditioning of its
// projections on the kept and discarded subspaces, typically 10..1000), so the
// tolerance sits three decades below the 1e-12 the angle itself should reach.  When
// every leaf has converged iws[done_slot] is set to 1 (it is never cleared here).
constexpr double kLeafConvTol = 1e-15;
constexpr int kLeafPowerCap = 6;
struct LeafCheck {
    int64_t sig_off;      // w singular values of the sketch (descending, zero padded)
    int32_t w;            // sketch width
    int32_t kcap, rule;   // the leaf's rank cap and truncation rule
    int32_t floor_rows, floor_cols;
    int32_t pad;
    double tol;
};
hipError_t launch_leaf_check(const double* ws, int* iws, const LeafCheck* items, int count, int step,
                             int done_slot, const int* guard, hipStream_t s);
// Per-execute state reset: flags[0..3] = 0 and iws[slots[i]] = 0 for i < nslots
// (a kernel, so that a captured graph holds no memset node).
hipError_t launch_reset_state(unsigned* flags, int* iws, const int* slots, int nslots, hipStream_t s);
// Output of `count` matrices (args: device array; ptrs: the pointer table);
// kmax, mmax, nmax bound k, m, n over the batch (grid sizes).
hipError_t launch_output(int fp32, const double* ws, int* iws, const OutputArgs* args, int count,
                         int kmax, int mmax, int nmax, void* const* ptrs, hipStream_t s);

}  // namespace hsvd
