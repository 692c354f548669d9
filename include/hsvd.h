/*
 * hsvd.h -- C ABI of the MI355X (gfx950) hierarchical merge-and-truncate SVD.
 *
 * Method: Vasudevan & Ramakrishna, "A Hierarchical Singular Value Decomposition
 * Algorithm for Low Rank Matrices" (arXiv:1710.02812), Section 3, Algorithm 1,
 * followed by the left-vector projection of Section 3 and optionally
 * Algorithm 2 (iterative improvement).
 *
 * Problem statement (Algorithm 1 inputs): a matrix X (m x n), a block grid and the
 * truncation parameter gamma.  Here the grid is given as counts: p row slabs and
 * q column slices; rows and columns are split as evenly as possible (the first
 * m mod p slabs one row taller, likewise columns).  gamma is `tol`; `k` caps
 * every kept rank (the fixed-rank variant of Section 3.1).  Outputs are the
 * approximate leading singular triplets: U (m x k), S (k), Vt (k x n).
 *
 * Conventions for every function:
 *   - Every call returns an hsvd_status; nothing throws across the ABI.
 *   - A non-OK return stores a message retrievable with hsvd_last_error()
 *     (thread-local, valid until the next call on the same thread).
 *   - Argument errors are detected on the host, return HSVD_ERR_INVALID and
 *     have no side effects.
 *   - Pointers named A, U, S, Vt are DEVICE pointers owned by the caller
 *     (e.g. torch tensor data pointers on the ROCm device).  Pointers ending in
 *     _host are host pointers owned by the caller.
 *   - A plan owns the device workspace it allocates at plan time and frees it in
 *     hsvd_destroy.  Plans are immutable after creation; one plan must not run
 *     on two streams at once.
 */
#ifndef HSVD_H
#define HSVD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsvd_plan_st* hsvd_plan_t;

typedef enum {
    HSVD_OK = 0,
    HSVD_ERR_INVALID = 1,      /* bad argument (host-side check; no side effects)      */
    HSVD_ERR_ALLOC = 2,        /* device or host allocation failed                      */
    HSVD_ERR_HIP = 3,          /* a HIP runtime call failed (see hsvd_last_error)       */
    HSVD_ERR_NONFINITE = 4,    /* reserved: reported through hsvd_get_status flags      */
    HSVD_ERR_NOCONV = 5,       /* reserved: reported through hsvd_get_status flags      */
    HSVD_ERR_UNSUPPORTED = 6   /* valid request this build does not implement           */
} hsvd_status;

/* Storage and arithmetic of the passes over A.
 *   FP64: A, U, S, Vt are double; all arithmetic float64.
 *   FP32: A, U, S, Vt are float (float32 storage); the products with A read
 *         float32 and run in float64 arithmetic, as does everything else.
 *   MIXED_BF16: A, U, S, Vt are float.  The leaf passes and the slab
 *         re-projection run on the matrix cores with A and the panels rounded to
 *         bfloat16 and float32 sums; the projection and one iteration of
 *         Algorithm 2 (always added; refine_steps counts further ones) read the
 *         float32 A unrounded on the float32 matrix cores (panels rounded to
 *         float32, float32 sums), so S and the subspaces are refined against the
 *         unrounded input to float32 accuracy.  Factor panels, QR and the Jacobi
 *         cores are float64 throughout.                                         */
typedef enum { HSVD_FP64 = 0, HSVD_FP32 = 1, HSVD_MIXED_BF16 = 2 } hsvd_precision;

/* Truncation rule (Section 3): GAMMA keeps s_i >= tol * s_1 of the matrix being
 * truncated; FROB keeps the shortest prefix whose discarded energy
 * sum_{i>=r} s_i^2 is <= tol^2 * sum_i s_i^2.  Both cap r <= k and drop values at
 * or below the numerical-zero floor max(rows, cols) * 2^-52 * s_1.              */
typedef enum { HSVD_RULE_GAMMA = 0, HSVD_RULE_FROB = 1 } hsvd_rule;

typedef struct {
    int32_t  precision;     /* hsvd_precision, default HSVD_FP64                        */
    int32_t  rule;          /* hsvd_rule, default HSVD_RULE_GAMMA                       */
    int32_t  oversample;    /* leaf sketch width l = k + oversample (capped by the block
                               sides), default 14                                       */
    int32_t  power_steps;   /* power steps per leaf (each one product with A_b^T and one
                               with A_b after the sketch Y = A_b Omega), 0..64, or -1
                               (default): float64 plans iterate until converged -- after
                               step t the leaf core gives the sketch's singular values
                               s_0..s_{l-1}, and with r the leaf's truncation rank the
                               step count is enough once (s_{l-1} / s_{r-1})^(2t+1) <= 1e-15
                               for every leaf (the subspace-iteration bound on how far a
                               further step could turn the kept subspace), at most 6
                               steps; float32, mixed and width plans take 1 step for -1 */
    int32_t  refine_steps;  /* iterations of Algorithm 2 after the projection, default 0 */
    int32_t  max_sweeps;    /* Jacobi sweep cap per core, default 40                    */
    uint64_t seed;          /* seed of the leaves' Gaussian test matrices, default 0    */
    double   refine_eps;    /* Algorithm 2 to a tolerance, default 0 (off).  When > 0 and
                               at least two iterations are asked for, the iterations stop
                               after the first t >= 1 at which, for every matrix of the plan,
                               ||s_t - s_(t-1)||_2 <= refine_eps ||s_(t-1)||_2 over its rank
                               (s_t: singular values after iteration t; s_0: Algorithm 1's,
                               the root of the row-slab tree); refine_steps (plus the mixed
                               path's own iteration) is then the cap and the output is
                               iteration t's.  Each test is taken on the device; the execute
                               then waits for it (one 4-byte read-back per iteration, the
                               last excepted), and per-launch timing (hsvd_set_profiling) is
                               refused.  Must not be negative or NaN (HSVD_ERR_INVALID).  */
    int32_t  graph;         /* 1 (default): the first execute captures the plan's launch
                               sequence into a hipGraph (on a stream private to the plan)
                               and every execute launches that graph on the caller's
                               stream; 0: every execute launches its kernels one by one.
                               Plans stopped on refine_eps and executes with per-launch
                               timing on always launch one by one.                      */
    int32_t  order;         /* order of the two sets of merges (Section 3): HSVD_ORDER_ROWS_LAST
                               runs Algorithm 1 as printed (column merges inside each row
                               slab, then the row-slab tree: right vectors from the trees,
                               left ones by projection); HSVD_ORDER_COLS_LAST the opposite
                               order (row merges inside each column slab, then the
                               column-slab tree: left vectors from the trees, right ones by
                               projection); HSVD_ORDER_AUTO (default) picks COLS_LAST for a
                               single matrix with m < n, so that the last tree and the
                               projection run on the shorter side, else ROWS_LAST.  Width
                               and feature plans are always ROWS_LAST.                  */
    int32_t  thin_rows;     /* rows per chunk of the thin-panel products of the merges
                               (partial Grams C = X^T Y, their sums, Y - X C): 0 (default:
                               128) or a multiple of 64 in 64..1024.  Fewer, taller chunks
                               mean fewer partial sums and fewer work-groups.           */
    int32_t  merge_qr;      /* QR of the merge complements: bit 0 set, the column-merge
                               levels (the first tree) factor them by the one-launch
                               panel QR (one work-group per panel) instead of the
                               multi-work-group Cholesky QR; bit 1, the same for the
                               row-merge levels.  Default 0.                             */
    int32_t  leaf_qr;       /* QR of the leaves' sketch and power panels: 0 (default) the
                               one-launch panel QR when a launch has >= 128 panels, else
                               the chunked Householder TSQR; 1 always the panel QR; 2
                               always the TSQR.                                          */
    int32_t  autotune;      /* 1: hsvd_plan_ex / hsvd_plan_batched / hsvd_plan_gram choose
                               leaf_qr, thin_rows and merge_qr themselves: each candidate plan
                               executes on a Gaussian input of the plan's shapes (three
                               timed executes after a warm-up, the median compared), one
                               tunable at a time starting from the defaults, the fastest
                               kept.  The choice is cached for the process under a key of
                               the shapes, grid, k, options and device, and appended to
                               the file named by the environment variable HSVD_TUNE_CACHE
                               (read at the first autotuned plan) when it is set.  Needs
                               device memory for the candidates and the input while the
                               plan is made; its results are those of a plan made with the
                               chosen values.  Default 0.                               */
} hsvd_options;

#define HSVD_ORDER_AUTO 0
#define HSVD_ORDER_ROWS_LAST 1
#define HSVD_ORDER_COLS_LAST 2

/* Status flags read by hsvd_get_status (bit set = condition seen in the last execute). */
#define HSVD_FLAG_NONFINITE 0x1u   /* a core matrix held NaN or Inf                        */
#define HSVD_FLAG_NOCONV    0x2u   /* a Jacobi core hit max_sweeps before convergence      */
#define HSVD_FLAG_RANK_FALLBACK 0x4u /* a leaf of a width plan left more than tol^2 of its
                                       block's energy outside its sketch (see
                                       hsvd_get_leaf_info)                               */

/* Fills *opt with the defaults listed above. */
hsvd_status hsvd_default_options(hsvd_options* opt);

/* Creates a plan for an m x n input on a p x q grid, rank cap k, truncation tol.
 *   Requires 1 <= p <= m, 1 <= q <= n, 1 <= k <= min(m, n), 0 <= tol < 1, out != NULL.
 *   k may exceed a block side: leaf ranks are capped by min(block rows, block cols).
 *   HSVD_ERR_UNSUPPORTED for k > 80 (the merge cores of this build hold 2k <= 160
 *   columns; the leaves' sketch width is at most 80 columns).
 *   Allocates the device workspace on the current HIP device and generates the
 *   leaves' Gaussian test matrices there (synchronously).  Uses default options. */
hsvd_status hsvd_plan(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q,
                      int32_t k, double tol);

/* As hsvd_plan with explicit options (opt == NULL means defaults). */
hsvd_status hsvd_plan_ex(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q,
                         int32_t k, double tol, const hsvd_options* opt);

/* Runs the method on A and writes the result.  Asynchronous, ordered on `stream`
 * (0 = the null stream); no host synchronisation inside, except the waits of
 * Algorithm 2 stopped on refine_eps (see hsvd_options) and a wait for the previous
 * execute when the data pointers differ from its (the device pointer table is
 * replaced).  With opt.graph = 1 the first execute captures the launches into a
 * hipGraph and every execute replays it (the graph reads A, U, S, Vt through the
 * pointer table, so one graph serves every input).
 *   A  : m x n, row-major, contiguous (leading dimension n), read only.
 *   U  : m x k, row-major.   S : k, descending.   Vt : k x n, row-major.
 *   Element type double (FP64 plans) or float (FP32 plans).
 *   The effective rank r <= k is kept on the device (hsvd_get_rank); columns of U,
 *   entries of S and rows of Vt at index >= r are written as zero.
 *   Signs: each column u_i has its largest-magnitude entry positive (ties: lowest
 *   row index), with v_i flipped alike.
 *   A, U, S, Vt must not overlap.                                               */
hsvd_status hsvd_execute(hsvd_plan_t plan, const void* A, void* U, void* S, void* Vt,
                         hipStream_t stream);
/* (A plan from hsvd_plan_batched takes hsvd_execute_batched instead.) */

/* Plan over `count` matrices of arbitrary shapes (Section 3: the leaves and the
 * merges of different matrices are independent), executed together: every launch
 * of an execute covers the same stage of all matrices.  m[i], n[i], p[i], q[i],
 * k[i] (host arrays) describe matrix i with the same constraints as hsvd_plan_ex;
 * tol and opt apply to all.  Each matrix keeps its own rank cap k[i] and takes its own
 * sketch width (k[i] + oversample, rounded up to a multiple of 8, at most 80); the
 * matrices are grouped into at most 4 rank classes of adjacent sketch widths, each
 * class running its whole pipeline with the panel width of its largest k[i], the
 * classes concurrently (a batch stopping Algorithm 2 on refine_eps runs as one class).
 * HSVD_ERR_INVALID names the first bad matrix; count must be 1..65535.         */
hsvd_status hsvd_plan_batched(hsvd_plan_t* out, int32_t count, const int64_t* m, const int64_t* n,
                              const int32_t* p, const int32_t* q, const int32_t* k, double tol,
                              const hsvd_options* opt);

/* Execute of a plan from hsvd_plan_batched: A[i], U[i], S[i], Vt[i] (host arrays
 * of device pointers) are the operands of matrix i, laid out as in hsvd_execute.
 * Asynchronous on `stream`; when the pointers differ from the previous execute's,
 * the call first waits for the previous execute and uploads the new pointers.   */
hsvd_status hsvd_execute_batched(hsvd_plan_t plan, const void* const* A, void* const* U,
                                 void* const* S, void* const* Vt, hipStream_t stream);

/* Plan for the SVD of X (m x n) through its Gram matrix (Section 4 results: the method
 * applied to X^T X): each execute forms G = X^T X (n x n, float64 matrix cores, float64
 * sums, held in the plan's workspace), runs the method on G with a p x q grid of G
 * (1 <= p, q <= n; tol and the rule apply to G's singular values, which are X's
 * squared), takes V-hat from G's row-slab tree (G's right singular vectors are X's) and
 * projects X itself onto it (Section 3: SVD(X V-hat)), so that U, S and Vt are X's:
 * U (m x k), S (k), Vt (k x n), as hsvd_execute.  refine_steps run Algorithm 2 on X.
 * Execute with hsvd_execute.  Options as hsvd_plan_ex; MIXED_BF16 and batched use are
 * HSVD_ERR_UNSUPPORTED; order is ignored (G is square).  The workspace holds G (and, for
 * tall X, n^2-sized partial sums of up to ceil(1024 / tiles) row chunks).            */
hsvd_status hsvd_plan_gram(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                           double tol, const hsvd_options* opt);

/* Frees the plan and its workspace after synchronising its last stream.
 * plan == NULL is accepted and does nothing. */
hsvd_status hsvd_destroy(hsvd_plan_t plan);

/* Copies the effective rank of the last execute to *r_host (synchronises that
 * execute's stream).  Single-matrix plans only. */
hsvd_status hsvd_get_rank(hsvd_plan_t plan, int32_t* r_host);

/* Iterations of Algorithm 2 (Section 3, iterative improvement) that the last execute
 * of an SVD plan ran into its output: refine_steps (plus one on the mixed path) unless
 * refine_eps stopped them earlier.  Host-side value, no synchronisation.
 * HSVD_ERR_INVALID for NULL arguments or a block-feature plan.                    */
hsvd_status hsvd_get_refine_iterations(hsvd_plan_t plan, int32_t* iters_host);

/* Effective ranks of all `count` matrices of the last execute (count must equal
 * the plan's matrix count; synchronises). */
hsvd_status hsvd_get_ranks(hsvd_plan_t plan, int32_t* r_host, int32_t count);

/* Copies the status of the last execute to *flags_host (synchronises): bits 0..15
 * hold the HSVD_FLAG_* conditions, bits 16..31 the largest number of Jacobi sweeps
 * any core of that execute ran. */
hsvd_status hsvd_get_status(hsvd_plan_t plan, uint32_t* flags_host);

/* The thin_rows, merge_qr and leaf_qr a plan runs with (thin_rows resolved: 128 when
 * 0), whether they came from the autotuner (*tuned = 1), and then the median execute
 * time (ms) of the chosen candidate during tuning.  Any pointer may be NULL.  Host
 * only.                                                                           */
hsvd_status hsvd_get_tuning(hsvd_plan_t plan, int32_t* thin_rows, int32_t* merge_qr, int32_t* leaf_qr,
                            int32_t* tuned, float* tuned_ms);

/* Bytes of the plan's device workspace: its float64 arena (panels, scratch, the
 * leaves' Gaussian test matrices) and its int arena (ranks, counters, flags), as
 * hsvd_set_workspace lays them out.  The task tables and the pointer table (a few
 * hundred KB at most) are not included. */
hsvd_status hsvd_workspace_bytes(hsvd_plan_t plan, size_t* bytes_host);

/* Moves the plan's workspace (see hsvd_workspace_bytes) into a caller-owned device
 * buffer, e.g. memory from PyTorch's caching allocator: the current contents are copied
 * there and the plan's own allocation is freed; later executes use the buffer.
 *   dptr: device pointer on the plan's device, 256-byte aligned; bytes >= the value
 *   hsvd_workspace_bytes reports.  The caller keeps ownership and must keep the buffer
 *   alive and untouched until hsvd_destroy (or a later hsvd_set_workspace).
 *   Synchronises the plan's last stream.  A captured graph is discarded (the next
 *   execute captures again).  HSVD_ERR_INVALID for NULL, misaligned or short buffers
 *   (the message gives the bytes needed) and for no side effects in that case.        */
hsvd_status hsvd_set_workspace(hsvd_plan_t plan, void* dptr, size_t bytes);

/* Launch kinds reported by hsvd_launch_times. */
typedef enum {
    HSVD_LAUNCH_GEMM_AX = 0,       /* Y = A_blk X   (passes over A)                      */
    HSVD_LAUNCH_GEMM_ATX = 1,      /* Y = A_blk^T X (passes over A)                      */
    HSVD_LAUNCH_TSQR_FACTOR = 2,   /* Householder TSQR of panels                         */
    HSVD_LAUNCH_TSQR_APPLY = 3,    /* Q X from the TSQR factors                          */
    HSVD_LAUNCH_GRAM = 4,          /* projection coefficients X^T Y (row-chunk partials) */
    HSVD_LAUNCH_REDUCE = 5,        /* sum of the partials                                */
    HSVD_LAUNCH_THIN_NN = 6,       /* Y (+/-)= X C                                       */
    HSVD_LAUNCH_SUM = 7,           /* sum of split products                              */
    HSVD_LAUNCH_CORE = 8,          /* Jacobi SVD cores                                   */
    HSVD_LAUNCH_OUTPUT = 9,        /* signs and the U, S, Vt writes                      */
    HSVD_LAUNCH_GEMM_AX_BF16 = 10, /* Y = A_blk X on the bfloat16 matrix cores           */
    HSVD_LAUNCH_GEMM_ATX_BF16 = 11,/* Y = A_blk^T X on the bfloat16 matrix cores         */
    HSVD_LAUNCH_ENERGY = 12,       /* squared Frobenius norms of the blocks              */
    HSVD_LAUNCH_FEATURES = 13,     /* block features of a feature plan                   */
    HSVD_LAUNCH_CHOLQR = 14,       /* Cholesky QR passes (fast path of the panel QRs)    */
    HSVD_LAUNCH_CHECK = 15,        /* the leaves' power-step convergence test            */
    HSVD_LAUNCH_PANEL_QR = 16,     /* leaf panels: repeated Cholesky QR, one group each  */
    HSVD_LAUNCH_GEMM_AX_F32 = 17,  /* Y = A_blk X on the float32 matrix cores (mixed)    */
    HSVD_LAUNCH_GEMM_ATX_F32 = 18, /* Y = A_blk^T X on the float32 matrix cores (mixed)  */
    HSVD_LAUNCH_GRAM_XTX = 19,     /* G = X^T X of a Gram plan (float64 matrix cores)    */
    HSVD_LAUNCH_CORE_WIDE = 20     /* Jacobi SVD of merge cores above 128 columns        */
} hsvd_launch_kind;

/* Turns per-launch timing on (1) or off (0) for later executes of this plan.
 * When on, execute records a HIP event on its stream after every launch. */
hsvd_status hsvd_set_profiling(hsvd_plan_t plan, int32_t enable);

/* Per-launch durations (ms) of the last profiled execute, in launch order:
 * kinds_host[i] (hsvd_launch_kind) and ms_host[i] for i < min(cap, count).
 * *count_host receives the number of launches of one execute; with
 * kinds_host == NULL or ms_host == NULL only the count is returned.
 * Synchronises on the last event. */
hsvd_status hsvd_launch_times(hsvd_plan_t plan, int32_t* kinds_host, float* ms_host, int32_t cap,
                              int32_t* count_host);

/* Algorithmic work of every launch of one execute, in the order of
 * hsvd_launch_times (host only, no device work): flops_host[i] and the minimal
 * HBM bytes bytes_host[i] (each operand read once, each result written once) for
 * i < min(cap, count).  Counts at the plan's rank caps (data-dependent ranks
 * can only lower them):
 *   passes over A        2 rows cols N flops per block and product width N;
 *   Householder TSQR     2 h w^2 - 2 w^3 / 3 per h x w panel;
 *   applying Q           4 h w c per panel and c columns;
 *   thin products        2 h wx wy;  sums of partials one flop per addend;
 *   SVD cores            22 n^3 per n x n core, the cost the paper's complexity
 *                        analysis gives a dense SVD (Section 3.1: 6 m n^2 + 16 n^3
 *                        at m = n, i.e. 176 k^3 for a 2k x 2k merge core).
 * *count_host receives the number of launches; with flops_host == NULL or
 * bytes_host == NULL only the count is returned. */
hsvd_status hsvd_launch_work(hsvd_plan_t plan, double* flops_host, double* bytes_host, int32_t cap,
                             int32_t* count_host);

/* ---------------------------------------------------------------- learned rank
 * A small network predicts, from a cheap sketch of each block, the rank the
 * tolerance rule would keep there, so that a leaf computes only the sketch columns
 * it needs (widths of a width plan).  The tolerance rule stays the judge: each
 * leaf of a width plan checks the energy its sketch missed and reports it.
 *
 * Features of block b (16 floats): with s_1 >= ... >= s_16 the singular values of
 * Y = A_b Omega (Omega a 16-column Gaussian test matrix) and E = ||A_b||_F^2:
 *   f_j = max(log10(s_{j+1} / s_1), -16) for j = 1..15,  f_16 = log10(16 E / sum s^2);
 * all zero for a zero block.
 * Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2) (64 units each),
 * y = w3 . h2 + b3 = predicted log2(rank); weights used rounded to float16,
 * float32 arithmetic.  Parameters (HSVD_RANK_MODEL_PARAMS floats): W1 (64 x 16
 * row-major) | b1 (64) | W2 (64 x 64 row-major) | b2 (64) | w3 (64) | b3 (1).     */
#define HSVD_RANK_FEATURES 16
#define HSVD_RANK_MODEL_PARAMS 5313
typedef struct hsvd_rank_model_st* hsvd_rank_model_t;

/* Feature plan for an m x n matrix on a p x q grid (precision FP64 or FP32 for A;
 * seed fixes Omega).  Execute with hsvd_features_execute only.                   */
hsvd_status hsvd_features_plan(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q,
                               int32_t precision, uint64_t seed);
/* features: device float array of p * q * 16, block (i, j) at row i * q + j. */
hsvd_status hsvd_features_execute(hsvd_plan_t plan, const void* A, float* features,
                                  hipStream_t stream);

/* A plan like hsvd_plan_ex whose leaves use per-block sketch widths:
 * leaf_width[i * q + j] (host array, each in 1..80) columns for block (i, j)
 * instead of k + oversample.  Its leaves also check the energy their sketch
 * missed (status bit HSVD_FLAG_RANK_FALLBACK, per block via hsvd_get_leaf_info):
 * a block whose missed share exceeds tol^2 (tol with the FROB rule) needs a wider
 * sketch.                                                                        */
hsvd_status hsvd_plan_widths(hsvd_plan_t* out, int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                             double tol, const hsvd_options* opt, const int32_t* leaf_width);

/* Per-block leaf ranks and fallback flags (1 = the sketch missed too much energy;
 * always 0 outside width plans) of the last execute of a single-matrix plan;
 * count = p * q; either output may be NULL.  Synchronises.                      */
hsvd_status hsvd_get_leaf_info(hsvd_plan_t plan, int32_t* ranks, int32_t* fallback, int32_t count);

/* Network with He-initialised weights (seeded) and a fresh Adam state. */
hsvd_status hsvd_rank_model_create(hsvd_rank_model_t* out, uint64_t seed);
hsvd_status hsvd_rank_model_destroy(hsvd_rank_model_t model);
/* Host copies of the float32 master parameters (count = HSVD_RANK_MODEL_PARAMS);
 * set also resets the Adam state and the minibatch counter.                     */
hsvd_status hsvd_rank_model_set_params(hsvd_rank_model_t model, const float* params_host, int32_t count);
hsvd_status hsvd_rank_model_get_params(hsvd_rank_model_t model, float* params_host, int32_t count);
/* `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8, rate lr) on the mean of
 * (y - t)^2 / 2 over minibatches of 64: step s of the model's life takes samples
 * (s * 64 + i) mod count.  X: count x 16 features, T: count log2-rank targets
 * (device).  losses (device, may be NULL) receives each step's minibatch loss.
 * Runs on the GPU in one work-group; asynchronous.                              */
hsvd_status hsvd_rank_model_train(hsvd_rank_model_t model, const float* X, const float* T, int32_t count,
                                  int32_t steps, float lr, float* losses, hipStream_t stream);
/* Gradient (device, HSVD_RANK_MODEL_PARAMS) and loss (device, 1) of minibatch
 * batch_index at the current weights, without updating anything.                 */
hsvd_status hsvd_rank_model_grad(hsvd_rank_model_t model, const float* X, const float* T, int32_t count,
                                 int32_t batch_index, float* grad, float* loss, hipStream_t stream);
/* out[i] = predicted log2(rank) of feature row i (device arrays). */
hsvd_status hsvd_rank_model_predict(hsvd_rank_model_t model, const float* X, int32_t count, float* out,
                                    hipStream_t stream);

/* Allocation-free one-shot SVD, for callers that cannot allocate device memory (code
 * that must not call hipMalloc: graph capture, tight serving loops, harnesses that
 * forbid it).  Same method, arguments and results as hsvd_plan_ex followed by
 * hsvd_execute on a single matrix (bit-identical outputs), but the plan's whole device
 * state -- arena, int arena, status flags, task tables and pointer table -- is placed
 * in a file-scope device array of 64 MiB (each GPU the library runs on holds its own
 * copy until the process ends) instead of hipMalloc'd memory; the schedule is built in
 * host memory.  The call clears the array with a kernel, uploads the task tables,
 * enqueues the method on `stream` and synchronises `stream` before it returns
 * (blocking); r_host (may be NULL) receives the effective rank.
 *   A, U, S, Vt: as hsvd_execute (device, caller-owned).
 *   Errors: as hsvd_plan_ex; HSVD_ERR_INVALID when the problem's device state exceeds
 *   64 MiB (about 1024^2 on a 4 x 4 grid with k = 32) -- the message gives the bytes it
 *   needs.  Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 *   (other threads, other streams) race and must be serialised by the caller.         */
hsvd_status hsvd_svd_static(int64_t m, int64_t n, int32_t p, int32_t q, int32_t k, double tol,
                            const hsvd_options* opt, const void* A, void* U, void* S, void* Vt,
                            int32_t* r_host, hipStream_t stream);

/* Attaches the rank model (weights_host: the HSVD_RANK_MODEL_PARAMS float32 parameters
 * in the layout above, bytes = 4 * HSVD_RANK_MODEL_PARAMS) to a single-matrix float64
 * or float32-storage plan; weights_host == NULL detaches it.  Later executes of the plan
 * take the learned path: the block features and the network's predictions are computed
 * on the device, each block's sketch width is ceil(2^prediction) + 8 rounded up to a
 * multiple of 8 (at most 80 and the block's sides), and a width plan (rebuilt only when
 * the widths change: an unseen input pays its creation) runs the method.  The tolerance
 * rule judges the result: a leaf whose sketch missed more than tol^2 of its block's
 * energy doubles its width and the call runs again (at most 3 times); if a leaf still
 * misses, the plan's own plain widths (k + oversample) compute the output.  Such
 * executes synchronise the stream (two read-backs per run).  hsvd_get_rank,
 * hsvd_get_status (bit HSVD_FLAG_RANK_FALLBACK: refits ran) and hsvd_get_leaf_info
 * report the run that produced the output; hsvd_get_leaf_widths the widths.
 * HSVD_ERR_INVALID for other plans or a wrong size; HSVD_ERR_UNSUPPORTED for mixed plans. */
hsvd_status hsvd_set_rank_model(hsvd_plan_t plan, const void* weights_host, size_t bytes);

/* After a learned execute: the p * q sketch widths of its last run (widths_host, count =
 * p * q; may be NULL), the refits it ran and whether the plain widths produced the
 * output (1) or the learned ones (0).  Host-side values, no synchronisation.          */
hsvd_status hsvd_get_leaf_widths(hsvd_plan_t plan, int32_t* widths_host, int32_t count, int32_t* refits_host,
                                 int32_t* plain_host);

/* Message for the last non-OK return on this thread ("" if none). */
const char* hsvd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HSVD_H */
