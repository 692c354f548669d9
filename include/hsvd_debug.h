/*
 * hsvd_debug.h -- kernel-level entry points of libhsvd for parity tests.
 *
 * They run one building block of the hierarchical SVD on caller data so that
 * each kernel can be checked against a CPU reference on its own.  Same
 * conventions as hsvd.h: hsvd_status returns, hsvd_last_error() messages,
 * device pointers owned by the caller, asynchronous on `stream`, float64
 * col-major matrices stored back to back for a batch.  Each call allocates and
 * frees its own scratch (it synchronises `stream` before freeing).
 */
#ifndef HSVD_DEBUG_H
#define HSVD_DEBUG_H
#include "hsvd.h"
#ifdef __cplusplus
extern "C" {
#endif

/* One-sided Jacobi SVD of `batch` dense n x n matrices M (n <= 160), the core
 * that every leaf, merge (Section 3, eqs. orthmerge1 and orthmerge) and
 * projection step of the hierarchical SVD runs on its small matrix: the
 * LDS-resident cores for n <= 128, the wide cores (columns in a global scratch
 * panel) above.  Writes the left singular vectors U (n x n, columns by descending
 * sigma), S (n, descending) and, when V != NULL (then n <= 96), the right singular
 * vectors V (n x n), so that M = U diag(S) V^T.  Columns with sigma = 0 are 0.
 * precondition = 1 first replaces M by L of M = L Q (left pairs only; V must be
 * NULL), as the merge cores do; 0 runs the sweeps on M itself.
 * *flags_host (may be NULL) receives the status flags (HSVD_FLAG_*) in bits 0..15
 * and the largest number of sweeps any core ran in bits 16..31.
 * HSVD_ERR_INVALID for null M/U/S, n outside 1..160, V with n > 96, max_sweeps < 1,
 * precondition not 0/1 or precondition with V.                            */
hsvd_status hsvd_debug_jacobi(const double* M, int32_t batch, int32_t n, double* U, double* S,
                              double* V, int32_t max_sweeps, int32_t precondition,
                              uint32_t* flags_host, hipStream_t stream);

/* One product of a pass over A on a single block, as the plans run it:
 * op 0: Y = A X with A rows x cols, X cols x N;  op 1: Y = A^T X with X rows x N.
 * kind 0: float64 arithmetic (A float64 when a_fp32 = 0, float32 otherwise);
 * kind 1: bfloat16 matrix cores (A float32, X rounded to float32 then bfloat16,
 * float32 sums; requires a_fp32 = 1); kind 2: float32 matrix cores (A float32 as
 * is, X rounded to float32, float32 sums; requires a_fp32 = 1).  A row-major with
 * leading dimension lda; X col-major (ld = its row count); Y col-major (ld = its
 * row count: rows for op 0, cols for op 1); 1 <= N <= 1024 (N <= 96 for kinds 1
 * and 2).  HSVD_ERR_INVALID on bad arguments. */
hsvd_status hsvd_debug_gemm(int32_t op, int32_t kind, int32_t a_fp32, const void* A, int64_t rows,
                            int64_t cols, int64_t lda, const double* X, int32_t N, double* Y,
                            hipStream_t stream);

/* Builds and bounds-checks a plan on the host only (no device work): every task
 * of every launch is checked against the workspace and A.  *workspace_bytes (may be
 * NULL) receives the float64 arena size.  Returns what hsvd_plan_ex would return
 * for the arguments, short of device allocation. */
hsvd_status hsvd_debug_plan_check(int64_t m, int64_t n, int32_t p, int32_t q, int32_t k,
                                  double tol, const hsvd_options* opt, size_t* workspace_bytes);

/* hsvd_debug_plan_check for a plan over `count` matrices (hsvd_plan_batched). */
hsvd_status hsvd_debug_plan_check_batched(int32_t count, const int64_t* m, const int64_t* n,
                                          const int32_t* p, const int32_t* q, const int32_t* k,
                                          double tol, const hsvd_options* opt,
                                          size_t* workspace_bytes);

/* Householder TSQR of `batch` h x w panels P (w <= 80): Q (h x w, orthonormal
 * columns) and R (w x w upper triangular) with P = Q R.  P is not modified.   */
hsvd_status hsvd_debug_tsqr(const double* P, int32_t batch, int64_t h, int32_t w, double* Q,
                            double* R, hipStream_t stream);

/* The tall-skinny QR as the merge, re-projection and projection panels take it
 * (w <= 64): two Cholesky QR passes (R1 = chol(P^T P), Q1 = P R1^-1, then the same on
 * Q1; R = R2 R1, Q = Q1 R2^-1), with the Householder TSQR in their place when the
 * first pass meets a pivot below 1e-10 of its column's squared norm or the second
 * finds ||Q1^T Q1 - I||_F > 1/4.  P (batch x h x w, each col-major with ld h, device)
 * is not modified; Q (same layout) and R (batch x w x w, col-major, upper triangular)
 * are written with P = Q R.  Exactly zero columns of P give zero rows of R and zero
 * columns of Q on the Cholesky path.  fell_back (host, batch ints) receives 1 where
 * the Householder kernels ran, else 0.  Errors: HSVD_ERR_INVALID for null pointers or
 * sizes out of range, HSVD_ERR_ALLOC, HSVD_ERR_HIP.                                   */
hsvd_status hsvd_debug_cholqr(const double* P, int32_t batch, int64_t h, int32_t w, double* Q,
                              double* R, int32_t* fell_back, hipStream_t stream);

/* The leaves' one-launch panel QR (repeated Cholesky QR in one work-group per panel,
 * the first pass shifted) on `batch` panels P (device, h x w col-major each, w <= 80),
 * with the Householder TSQR run where it falls back; Q (h x w) and R (w x w, upper)
 * as in hsvd_debug_tsqr, fell_back (host, batch ints) 1 where the Householder kernels
 * ran.  P is not modified.  Errors as hsvd_debug_cholqr.                             */
hsvd_status hsvd_debug_panel_qr(const double* P, int32_t batch, int64_t h, int32_t w, double* Q,
                                double* R, int32_t* fell_back, hipStream_t stream);

/* Peak probes of the device (measurement only, no part of the method): the rates a
 * plain kernel of this library reaches, beside which the method's kernels are read.
 *   kind 0: streams the first `bytes` of buf through 16-byte loads (HBM read rate);
 *   kind 1: copies the first half of those bytes onto the second half (read + write);
 *   kinds 2, 3, 4: every wave runs 4 independent accumulation chains of `iters`
 *   float64 16x16x4, bfloat16 16x16x32 (float32 sums) or float32 16x16x4 matrix-core
 *   instructions, 8 waves on every SIMD; buf is not used.
 * buf: device memory of at least `bytes` bytes, 16-byte aligned (kinds 0 and 1).
 * Blocks until the launch is done: *ms_host receives its duration (HIP events around
 * it on `stream`), *work_host the bytes moved (kinds 0, 1) or the flops (kinds 2-4).
 * Errors: HSVD_ERR_INVALID for null outputs, kind outside 0..4, bytes < 32 or an
 * unaligned buf (kinds 0, 1), iters outside 1..2^24 (kinds 2-4); HSVD_ERR_ALLOC,
 * HSVD_ERR_HIP.                                                                       */
hsvd_status hsvd_debug_probe(int32_t kind, void* buf, int64_t bytes, int32_t iters, double* ms_host,
                             double* work_host, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
