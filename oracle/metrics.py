"""Sign- and rotation-free comparison metrics for truncated SVD factors.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's accuracy report).

  * e_sigma: max_i |s_hat_i - s_i| / s_0.
  * sin_theta: largest principal-angle sine between two column spaces, in the
    sine form ||U_hat - U (U^T U_hat)||_2, which resolves angles far below the
    ~1.5e-8 limit of the arccos form in float64.
  * e_frob: ||U_h S_h V_h^T - U S V^T||_F / ||s||_2 evaluated in factored form,
    ||R_a R_b^T||_F with [U_h S_h, -U S] = Q_a R_a and [V_h, V] = Q_b R_b, so no
    m x n matrix is formed and differences near 1e-12 stay resolvable.
  * paper_error: the paper's ||X_k - X_hat_k||_F / ||X_k||_F (Section 4), X_k the
    LAPACK truncation of A at the same rank (small matrices only).
"""
from __future__ import annotations

import numpy as np


def e_sigma(s_hat, s) -> float:
    s_hat = np.asarray(s_hat, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    n = max(s_hat.size, s.size)
    a = np.zeros(n)
    b = np.zeros(n)
    a[:s_hat.size] = s_hat
    b[:s.size] = s
    if b.size == 0 or b[0] == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / b[0])


def sin_theta(U_hat, U) -> float:
    """Sine of the largest principal angle between span(U_hat) and span(U)."""
    U_hat = np.asarray(U_hat, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    if U.shape[1] == 0 and U_hat.shape[1] == 0:
        return 0.0
    if U.shape[1] != U_hat.shape[1]:
        return 1.0
    D = U_hat - U @ (U.T @ U_hat)
    return float(np.linalg.norm(D, 2))


def e_frob(U_h, s_h, V_h, U, s, V) -> float:
    """||U_h diag(s_h) V_h^T - U diag(s) V^T||_F / ||s||_2 in factored form."""
    U_h, s_h, V_h, U, s, V = (np.asarray(x, dtype=np.float64) for x in (U_h, s_h, V_h, U, s, V))
    Ra = np.linalg.qr(np.hstack([U_h * s_h, -U * s]), mode="r")
    Rb = np.linalg.qr(np.hstack([V_h, V]), mode="r")
    denom = np.linalg.norm(s)
    if denom == 0.0:
        denom = 1.0
    return float(np.linalg.norm(Ra @ Rb.T) / denom)


def amplification(s_full, r: int) -> float:
    """sigma_1 / (sigma_r - sigma_{r+1}) of the reference spectrum (subspace sensitivity)."""
    s_full = np.asarray(s_full, dtype=np.float64)
    nxt = s_full[r] if r < s_full.size else 0.0
    gap = s_full[r - 1] - nxt
    return float(np.inf if gap <= 0 else s_full[0] / gap)


def paper_error(A, U_h, s_h, Vt_h, r: int) -> float:
    """||X_r - X_hat_r||_F / ||X_r||_F with X_r the LAPACK rank-r truncation of A."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    return e_frob(U_h[:, :r], s_h[:r], Vt_h[:r].T, U[:, :r], s[:r], Vt[:r].T)


def compare(U_h, s_h, Vt_h, r_h, U, s, Vt, r) -> dict:
    """All metrics between a candidate (U_h, s_h, Vt_h, r_h) and a reference (U, s, Vt, r)."""
    Vh = np.asarray(Vt_h, dtype=np.float64)[:r_h].T
    V = np.asarray(Vt, dtype=np.float64)[:r].T
    return {
        "rank_hat": int(r_h),
        "rank": int(r),
        "e_sigma": e_sigma(np.asarray(s_h)[:r_h], np.asarray(s)[:r]),
        "sin_u": sin_theta(np.asarray(U_h)[:, :r_h], np.asarray(U)[:, :r]),
        "sin_v": sin_theta(Vh, V),
        "e_frob": e_frob(np.asarray(U_h)[:, :r_h], np.asarray(s_h)[:r_h], Vh,
                         np.asarray(U)[:, :r], np.asarray(s)[:r], V),
    }
