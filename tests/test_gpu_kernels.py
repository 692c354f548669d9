"""Kernel-level parity on the GPU: the Jacobi core and the TSQR kernels through
the C ABI's debug entry points, against LAPACK on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1710_02812_amd import hsvd as H  # noqa: E402

DEV = "cuda:0"


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64, 80, 90, 96, 100, 128])
def test_jacobi_dense_random(n):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((3, n, n))
    M[1] *= np.exp(-np.arange(n) / 3.0)[None, :]          # graded columns
    print(f"jacobi n={n}", flush=True)
    U, S, V, flags, sweeps = H.debug_jacobi(_t(M), with_v=(n <= 96))
    print(f'sweeps {sweeps}', flush=True)
    assert flags == 0
    U, S = U.cpu().numpy(), S.cpu().numpy()
    for b in range(3):
        s_ref = np.linalg.svd(M[b], compute_uv=False)
        assert np.max(np.abs(S[b] - s_ref)) <= 1e-13 * s_ref[0] * max(1, n / 8)
        assert np.all(np.diff(S[b]) <= 0)
        nz = S[b] > 1e-12 * S[b][0]
        Ub = U[b][:, nz]
        assert np.linalg.norm(Ub.T @ Ub - np.eye(nz.sum())) <= 1e-13 * n
        if n <= 96:
            # columns past the zero floor (max(rows, cols) 2^-52 sigma_1) are written as zero
            Vb = V.cpu().numpy()[b]
            pos = S[b] > 0.0
            assert np.all(Vb[:, ~pos] == 0.0)
            assert np.linalg.norm(Vb[:, pos].T @ Vb[:, pos] - np.eye(pos.sum())) <= 1e-13 * n
            rec = (U[b] * S[b]) @ Vb.T
            assert np.linalg.norm(rec - M[b]) <= 1e-13 * n * np.linalg.norm(M[b])


def _merge_matrix(rng, k, h=600, noise=1e-6):
    """E = [[S1, C S2], [0, R S2]] of a merge of two nodes that share most of
    their directions (Section 3, eq. orthmerge1), as the merge cores see it."""
    base = np.linalg.qr(rng.standard_normal((h, k)))[0]
    mix = np.linalg.qr(rng.standard_normal((k, k)))[0]
    U1 = base
    U2 = np.linalg.qr(base @ mix + noise * rng.standard_normal((h, k)))[0]
    s1 = np.exp(-np.arange(k) / 8.0)
    s2 = np.exp(-np.arange(k) / 8.0) * 0.9
    C = U1.T @ U2
    Q = U2 - U1 @ C
    C2 = U1.T @ Q
    Q -= U1 @ C2
    C += C2
    R = np.linalg.qr(Q, mode="r")
    E = np.zeros((2 * k, 2 * k))
    E[:k, :k] = np.diag(s1)
    E[:k, k:] = C * s2
    E[k:, k:] = R * s2
    return E


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64, 90, 100, 128])
def test_jacobi_preconditioned(n):
    """LQ-preconditioned sweeps: same singular values, orthonormal left vectors,
    U^T M has orthogonal rows of norms S (M M^T = U S^2 U^T)."""
    rng = np.random.default_rng(1000 + n)
    M = rng.standard_normal((3, n, n))
    M[1] *= np.exp(-np.arange(n) / 3.0)[None, :]
    M[2] = np.triu(M[2])
    print(f"jacobi lq n={n}", flush=True)
    U, S, _, flags, sweeps = H.debug_jacobi(_t(M), with_v=False, precondition=True)
    print(f"sweeps {sweeps}", flush=True)
    assert flags == 0
    U, S = U.cpu().numpy(), S.cpu().numpy()
    for b in range(3):
        s_ref = np.linalg.svd(M[b], compute_uv=False)
        assert np.max(np.abs(S[b] - s_ref)) <= 1e-13 * s_ref[0] * max(1, n / 8)
        nz = S[b] > 1e-12 * S[b][0]
        Ub = U[b][:, nz]
        assert np.linalg.norm(Ub.T @ Ub - np.eye(nz.sum())) <= 1e-13 * n
        B = Ub.T @ M[b]
        assert np.linalg.norm(B @ B.T - np.diag(S[b][nz] ** 2)) <= 1e-13 * n * s_ref[0] ** 2


@pytest.mark.parametrize("k", [20, 50, 64])
def test_jacobi_merge_matrix_preconditioned(k):
    """Merge-shaped cores: preconditioning gives the same pairs in fewer sweeps."""
    rng = np.random.default_rng(k)
    E = _merge_matrix(rng, k)[None]
    print(f"merge core k={k}", flush=True)
    U0, S0, _, f0, sw0 = H.debug_jacobi(_t(E), with_v=False)
    U1, S1, _, f1, sw1 = H.debug_jacobi(_t(E), with_v=False, precondition=True)
    print(f"sweeps plain {sw0} lq {sw1}", flush=True)
    assert f0 == 0 and f1 == 0
    s_ref = np.linalg.svd(E[0], compute_uv=False)
    S1 = S1.cpu().numpy()[0]
    assert np.max(np.abs(S1 - s_ref)) <= 1e-13 * s_ref[0] * 2 * k / 8
    assert sw1 < sw0
    # top-k left subspace against LAPACK (a gap separates it from the noise part)
    Ur = np.linalg.svd(E[0])[0][:, :k]
    Uk = U1.cpu().numpy()[0][:, :k]
    assert np.linalg.norm(Uk - Ur @ (Ur.T @ Uk), 2) <= 1e-11


@pytest.mark.parametrize("n", [129, 150, 160])
def test_jacobi_wide_dense(n):
    """Cores of more than 128 columns (columns in a global scratch panel, three-phase
    sweeps): singular values against LAPACK, orthonormal left vectors, and U^T M with
    orthogonal rows of norms S, on a random and a column-graded matrix."""
    rng = np.random.default_rng(n)
    M = rng.standard_normal((2, n, n))
    M[1] *= np.exp(-np.arange(n) / 6.0)[None, :]
    print(f"wide jacobi n={n}", flush=True)
    for pre in (False, True):
        U, S, _, flags, sweeps = H.debug_jacobi(_t(M), with_v=False, precondition=pre)
        print(f"precondition={pre} sweeps {sweeps}", flush=True)
        assert flags == 0
        _check_left_pairs(M, U.cpu().numpy(), S.cpu().numpy(), n)


def _check_left_pairs(M, U, S, n):
    for b in range(M.shape[0]):
        s_ref = np.linalg.svd(M[b], compute_uv=False)
        assert np.max(np.abs(S[b] - s_ref)) <= 1e-13 * s_ref[0] * n / 8
        assert np.all(np.diff(S[b]) <= 0)
        nz = S[b] > 1e-12 * S[b][0]
        Ub = U[b][:, nz]
        assert np.linalg.norm(Ub.T @ Ub - np.eye(nz.sum())) <= 1e-13 * n
        B = Ub.T @ M[b]
        assert np.linalg.norm(B @ B.T - np.diag(S[b][nz] ** 2)) <= 1e-13 * n * s_ref[0] ** 2


@pytest.mark.parametrize("k", [72, 80])
def test_jacobi_wide_merge_matrix(k):
    """Merge-shaped cores of 2k > 128 columns (two children of rank k sharing most of
    their directions) on the wide cores, plain and LQ-preconditioned: singular values
    and the top-k left subspace against LAPACK; preconditioning takes fewer sweeps."""
    rng = np.random.default_rng(k)
    E = _merge_matrix(rng, k)[None]
    s_ref = np.linalg.svd(E[0], compute_uv=False)
    Ur = np.linalg.svd(E[0])[0][:, :k]
    sweeps = []
    for pre in (False, True):
        U, S, _, f, sw = H.debug_jacobi(_t(E), with_v=False, precondition=pre)
        print(f"wide merge core k={k} precondition={pre} sweeps {sw}", flush=True)
        assert f == 0
        S = S.cpu().numpy()[0]
        assert np.max(np.abs(S - s_ref)) <= 1e-13 * s_ref[0] * 2 * k / 8
        Uk = U.cpu().numpy()[0][:, :k]
        assert np.linalg.norm(Uk - Ur @ (Ur.T @ Uk), 2) <= 1e-11
        sweeps.append(sw)
    assert sweeps[1] < sweeps[0]


def test_jacobi_wide_rank_deficient_zero_and_cap():
    """Wide cores on a rank-6 matrix, a zero matrix, and under a one-sweep cap."""
    rng = np.random.default_rng(7)
    n = 140
    A = rng.standard_normal((n, 6)) @ rng.standard_normal((6, n))
    Z = np.zeros((n, n))
    U, S, _, flags, _ = H.debug_jacobi(_t(np.stack([A, Z])), with_v=False)
    S = S.cpu().numpy()
    assert flags == 0
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(S[0] - s_ref)) <= 1e-12 * s_ref[0]
    assert np.all(S[1] == 0.0)
    assert np.all(U.cpu().numpy()[1] == 0.0)
    M = rng.standard_normal((1, n, n))
    _, _, _, flags, sweeps = H.debug_jacobi(_t(M), max_sweeps=1, with_v=False)
    assert sweeps == 1
    assert flags & H.FLAG_NOCONV


def test_jacobi_rank_deficient_and_zero():
    rng = np.random.default_rng(5)
    n = 40
    A = rng.standard_normal((n, 6)) @ rng.standard_normal((6, n))
    Z = np.zeros((n, n))
    U, S, V, flags, _ = H.debug_jacobi(_t(np.stack([A, Z])), with_v=True)
    S = S.cpu().numpy()
    assert flags == 0
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(S[0] - s_ref)) <= 1e-12 * s_ref[0]
    assert np.all(S[1] == 0.0)
    assert np.all(U.cpu().numpy()[1] == 0.0)


def test_jacobi_sweep_cap_flag():
    """A cap of one sweep on a random 64 x 64 matrix is reported, not hidden."""
    rng = np.random.default_rng(6)
    M = rng.standard_normal((1, 64, 64))
    _, _, _, flags, sweeps = H.debug_jacobi(_t(M), max_sweeps=1, with_v=False)
    assert sweeps == 1
    assert flags & H.FLAG_NOCONV


@pytest.mark.parametrize("h,w", [(1, 1), (5, 7), (64, 64), (100, 20), (1000, 50), (1024, 64),
                                 (257, 64), (3000, 80), (8192, 50), (4100, 64), (20000, 17)])
def test_tsqr_random_panels(h, w):
    rng = np.random.default_rng(h + w)
    P = rng.standard_normal((2, h, w))
    P[1, :, -1] = P[1, :, 0]                                # rank-deficient panel
    print(f"tsqr h={h} w={w}", flush=True)
    Q, R = H.debug_tsqr(_t(P))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    kk = min(h, w)
    for b in range(2):
        assert np.allclose(np.tril(R[b], -1), 0.0)
        assert np.linalg.norm(Q[b] @ R[b] - P[b]) <= 1e-13 * np.sqrt(h * w) * np.linalg.norm(P[b])
        G = Q[b][:, :kk].T @ Q[b][:, :kk]
        assert np.linalg.norm(G - np.eye(kk)) <= 1e-13 * np.sqrt(h) * w
        if b == 0:
            Rref = np.linalg.qr(P[b], mode="r")
            assert np.allclose(np.abs(np.diag(R[b])[:kk]), np.abs(np.diag(Rref)[:kk]),
                               rtol=1e-11, atol=1e-12 * np.abs(Rref).max())


def _graded_panel(rng, h, w, kappa):
    U = np.linalg.qr(rng.standard_normal((h, w)))[0]
    V = np.linalg.qr(rng.standard_normal((w, w)))[0]
    return (U * np.logspace(0, -np.log10(kappa), w)) @ V.T


@pytest.mark.parametrize("h,w,kappa", [(100, 20, 1e3), (1000, 50, 5e3), (1024, 64, 1e4), (257, 64, 10.0),
                                       (8192, 50, 1e3), (20000, 17, 1e2), (3000, 1, 1.0), (2048, 64, 1e5),
                                       (70000, 16, 1e3), (16641, 64, 1e2)])
def test_cholqr_well_conditioned(h, w, kappa):
    """Two Cholesky QR passes stand (no fallback) on panels of condition number up to
    1e5, with a float64 QR: P = Q R, Q orthonormal, R upper with P's singular values.
    Heights past 16384 rows (274 and 66 chunks of 256) sum the partial Grams up three
    levels of the fan-in-8 tree."""
    rng = np.random.default_rng(h + w)
    P = np.stack([_graded_panel(rng, h, w, kappa), rng.standard_normal((h, w))])
    print(f"cholqr h={h} w={w} kappa={kappa:g}", flush=True)
    Q, R, fb = H.debug_cholqr(_t(P))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert fb == [0, 0]
    for b in range(2):
        assert np.all(np.tril(R[b], -1) == 0.0)
        assert np.linalg.norm(Q[b] @ R[b] - P[b]) <= 1e-14 * np.sqrt(w) * np.linalg.norm(P[b])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(w)) <= 1e-14 * np.sqrt(h) * w
        s_ref = np.linalg.svd(P[b], compute_uv=False)
        assert np.max(np.abs(np.linalg.svd(R[b], compute_uv=False) - s_ref)) <= 1e-13 * s_ref[0]


def test_trees_with_many_panels_in_flight():
    """Many panels factored at once, so that the work-groups of every reduction tree
    (the TSQR R tree, wide 768-thread variant, and the Cholesky QR Gram tree) arrive
    from all XCDs concurrently: each panel still gives P = Q R with Q orthonormal."""
    rng = np.random.default_rng(77)
    for kind, (b, h, w) in (("tsqr", (48, 3000, 80)), ("cholqr", (64, 4096, 50))):
        P = rng.standard_normal((b, h, w))
        print(f"{kind} batch={b} h={h} w={w}", flush=True)
        if kind == "tsqr":
            Q, R = H.debug_tsqr(_t(P))
        else:
            Q, R, fb = H.debug_cholqr(_t(P))
            assert fb == [0] * b
        Q, R = Q.cpu().numpy(), R.cpu().numpy()
        res = np.linalg.norm(np.einsum("bij,bjk->bik", Q, R) - P, axis=(1, 2)) / np.linalg.norm(P, axis=(1, 2))
        orth = np.linalg.norm(np.einsum("bji,bjk->bik", Q, Q) - np.eye(w), axis=(1, 2))
        assert np.all(np.tril(R, -1) == 0.0) if kind == "cholqr" else np.allclose(np.tril(R, -1), 0.0)
        assert res.max() <= 1e-13, (kind, res.max())
        assert orth.max() <= 1e-13 * np.sqrt(h) * w, (kind, orth.max())


@pytest.mark.parametrize("h,w", [(600, 40), (5000, 64), (300, 7)])
def test_cholqr_fallback_and_dead_columns(h, w):
    """An ill-conditioned panel (a column within 1e-9 of its predecessors' span) falls
    back to the Householder kernels; exactly zero columns stay on the Cholesky path as
    zero rows of R and zero columns of Q; a panel wider than tall falls back too."""
    rng = np.random.default_rng(10 * h + w)
    good = rng.standard_normal((h, w))
    bad = rng.standard_normal((h, w))
    bad[:, -1] = bad[:, 0] + 1e-9 * rng.standard_normal(h)
    dead = rng.standard_normal((h, w))
    dead[:, [1, w // 2]] = 0.0
    P = np.stack([good, bad, dead])
    print(f"cholqr fallback h={h} w={w}", flush=True)
    Q, R, fb = H.debug_cholqr(_t(P))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert fb == [0, 1, 0]
    for b in range(3):
        assert np.allclose(np.tril(R[b], -1), 0.0)
        assert np.linalg.norm(Q[b] @ R[b] - P[b]) <= 1e-13 * np.sqrt(h * w) * np.linalg.norm(P[b])
    live = np.ones(w, bool)
    live[[1, w // 2]] = False
    assert np.all(Q[2][:, ~live] == 0.0) and np.all(R[2][~live, :] == 0.0)
    Ql = Q[2][:, live]
    assert np.linalg.norm(Ql.T @ Ql - np.eye(live.sum())) <= 1e-14 * np.sqrt(h) * w
    s_ref = np.linalg.svd(P[2], compute_uv=False)
    assert np.max(np.abs(np.linalg.svd(R[2], compute_uv=False) - s_ref)) <= 1e-13 * s_ref[0]
    Pw = rng.standard_normal((1, 5, 9))
    Qw, Rw, fbw = H.debug_cholqr(_t(Pw))
    assert fbw == [1]
    assert np.linalg.norm(Qw.cpu().numpy()[0] @ Rw.cpu().numpy()[0] - Pw[0]) <= 1e-13 * np.linalg.norm(Pw[0])


@pytest.mark.parametrize("h,w,kappa", [(1024, 78, 1e2), (1024, 78, 1e7), (1000, 33, 1e12), (257, 80, 1e4),
                                       (64, 16, 1.0), (4096, 64, 1e9), (130, 1, 1.0), (1024, 80, 1e13)])
def test_panel_qr(h, w, kappa):
    """The leaves' one-launch panel QR (repeated Cholesky QR, the first pass shifted)
    stands without the Householder fallback on panels of condition number up to 1e13:
    P = Q R, Q orthonormal, R upper triangular with P's singular values (absolute error
    1e-13 s_1, what a backward-stable QR gives)."""
    rng = np.random.default_rng(h * 7 + w)
    P = np.stack([_graded_panel(rng, h, w, kappa), rng.standard_normal((h, w))])
    print(f"panel qr h={h} w={w} kappa={kappa:g}", flush=True)
    Q, R, fb = H.debug_panel_qr(_t(P))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert fb == [0, 0]
    for b in range(2):
        assert np.all(np.tril(R[b], -1) == 0.0)
        assert np.linalg.norm(Q[b] @ R[b] - P[b]) <= 1e-14 * np.sqrt(w) * np.linalg.norm(P[b])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(w)) <= 1e-14 * np.sqrt(h) * w
        s_ref = np.linalg.svd(P[b], compute_uv=False)
        assert np.max(np.abs(np.linalg.svd(R[b], compute_uv=False) - s_ref)) <= 1e-13 * s_ref[0]


def test_panel_qr_fallback_dead_columns_and_many_panels():
    """An exactly rank-deficient panel (rank 5 of 20 columns: the sketch of an exactly
    low-rank block) falls back to the Householder kernels; exactly zero columns stay on
    the Cholesky path as zero columns of Q and zero rows of R; a zero panel gives Q = 0,
    R = 0; 256 leaf-shaped panels (1024 x 78) in one launch all stand."""
    rng = np.random.default_rng(5)
    h, w = 700, 20
    low = rng.standard_normal((h, 5)) @ rng.standard_normal((5, w))
    dead = rng.standard_normal((h, w))
    dead[:, [0, 7]] = 0.0
    P = np.stack([low, dead, np.zeros((h, w))])
    Q, R, fb = H.debug_panel_qr(_t(P))
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert fb == [1, 0, 0]
    for b in range(3):
        assert np.allclose(np.tril(R[b], -1), 0.0)
        assert np.linalg.norm(Q[b] @ R[b] - P[b]) <= 1e-13 * np.sqrt(h * w) * max(np.linalg.norm(P[b]), 1.0)
    assert np.linalg.norm(Q[0].T @ Q[0] - np.eye(w)) <= 1e-13 * np.sqrt(h) * w
    live = np.ones(w, bool)
    live[[0, 7]] = False
    assert np.all(Q[1][:, ~live] == 0.0) and np.all(R[1][~live, :] == 0.0)
    Ql = Q[1][:, live]
    assert np.linalg.norm(Ql.T @ Ql - np.eye(live.sum())) <= 1e-14 * np.sqrt(h) * w
    assert np.all(Q[2] == 0.0) and np.all(R[2] == 0.0)
    b, h, w = 256, 1024, 78
    P = rng.standard_normal((b, h, w)) * np.logspace(0, -3, w)[None, None, :]
    print(f"panel qr batch={b} h={h} w={w}", flush=True)
    Q, R, fb = H.debug_panel_qr(_t(P))
    assert fb == [0] * b
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    res = np.linalg.norm(np.einsum("bij,bjk->bik", Q, R) - P, axis=(1, 2)) / np.linalg.norm(P, axis=(1, 2))
    orth = np.linalg.norm(np.einsum("bji,bjk->bik", Q, Q) - np.eye(w), axis=(1, 2))
    assert res.max() <= 1e-14 * np.sqrt(w), res.max()
    assert orth.max() <= 1e-14 * np.sqrt(h) * w, orth.max()


def _bf16(x):
    """Round to bfloat16 (nearest even) through float32, as the matrix-core passes do."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("rows,cols,op,N", [(300, 200, 0, 50), (1024, 1024, 0, 64), (1000, 130, 1, 17),
                                            (129, 257, 1, 64), (1024, 1024, 1, 50), (77, 33, 0, 96),
                                            (1024, 1024, 0, 78), (1024, 1024, 1, 78), (1031, 517, 0, 80),
                                            (517, 1031, 1, 80), (2048, 301, 1, 7)])
def test_gemm_bf16_matrix_cores(rows, cols, op, N):
    """bfloat16 MFMA pass: equals the float64 product of the bfloat16-rounded operands
    up to float32 summation error (this also fixes the MFMA lane layout)."""
    rng = np.random.default_rng(rows + cols + N)
    A = rng.standard_normal((rows, cols)).astype(np.float32)
    K = cols if op == 0 else rows
    X = rng.standard_normal((K, N))
    print(f"gemm bf16 {rows}x{cols} op{op} N={N}", flush=True)
    At = torch.tensor(A, device=DEV)
    Y = H.debug_gemm(At, _t(X), op=op, bf16=True).cpu().numpy()
    Ab, Xb = _bf16(A), _bf16(X)
    ref = (Ab @ Xb) if op == 0 else (Ab.T @ Xb)
    bound = (np.abs(Ab) @ np.abs(Xb)) if op == 0 else (np.abs(Ab).T @ np.abs(Xb))
    assert np.all(np.abs(Y - ref) <= 2.0 * K * 2.0 ** -24 * bound + 1e-30)
    # the float32 matrix-core kernel: the float64 product of A and the float32-rounded X
    # up to float32 summation error
    Y32 = H.debug_gemm(At, _t(X), op=op, f32=True).cpu().numpy()
    A64 = A.astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    ref32 = (A64 @ X32) if op == 0 else (A64.T @ X32)
    bound32 = (np.abs(A64) @ np.abs(X32)) if op == 0 else (np.abs(A64).T @ np.abs(X32))
    assert np.all(np.abs(Y32 - ref32) <= 2.0 * K * 2.0 ** -24 * bound32 + 1e-30)
    # and the float64-arithmetic kernel on the same float32 A is exact to float64 rounding
    Y64 = H.debug_gemm(At, _t(X), op=op, bf16=False).cpu().numpy()
    A64 = A.astype(np.float64)
    ref64 = (A64 @ X) if op == 0 else (A64.T @ X)
    assert np.max(np.abs(Y64 - ref64)) <= 1e-13 * np.max(np.abs(ref64)) * np.sqrt(K)


@pytest.mark.parametrize("N", [17, 64, 65, 78, 96, 97, 128])
@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("a64", [False, True])
def test_gemm_float64_passes_every_width(N, op, a64):
    """The float64 matrix-core pass over a block, across the width where one 64 x 96 tile
    replaces two 64-column tiles (65..96 columns: A read once): exact to float64 rounding
    against the host product, ragged rows and columns included."""
    rows, cols = 203, 141
    rng = np.random.default_rng(N + 7 * op + (11 if a64 else 0))
    A = rng.standard_normal((rows, cols))
    if not a64:
        A = A.astype(np.float32)
    K = cols if op == 0 else rows
    X = rng.standard_normal((K, N))
    print(f"gemm f64 op{op} N={N} a64={a64}", flush=True)
    Y = H.debug_gemm(torch.tensor(A, device=DEV), _t(X), op=op).cpu().numpy()
    A64 = A.astype(np.float64)
    ref = (A64 @ X) if op == 0 else (A64.T @ X)
    bound = (np.abs(A64) @ np.abs(X)) if op == 0 else (np.abs(A64).T @ np.abs(X))
    assert Y.shape == ref.shape
    assert np.all(np.abs(Y - ref) <= 2.0 * K * 2.0 ** -53 * bound + 1e-300)


def test_peak_probes_are_plausible():
    """The library's peak probes: each reports the work it did and a rate below the
    device's published peak (HBM 8 TB/s; float64, bfloat16, float32 matrix cores 78.6,
    2500, 157.3 TFLOP/s), and above a tenth of it."""
    buf = torch.ones(64 << 20, dtype=torch.float32, device=DEV)       # 256 MiB
    for kind, peak in (("read", 8e12), ("copy", 8e12), ("mfma_f64", 78.6e12),
                       ("mfma_bf16", 2500e12), ("mfma_f32", 157.3e12)):
        mem = kind in ("read", "copy")
        H.debug_probe(kind, buf if mem else None, 0 if mem else 256)      # warm-up
        ms, work = H.debug_probe(kind, buf if mem else None, 0 if mem else 2048)
        rate = work / (ms * 1e-3)
        print(f"probe {kind}: {rate / 1e12:.2f} T/s", flush=True)
        if mem:                  # read streams the buffer; copy reads one half, writes the other
            assert work == buf.numel() * 4
        assert 0.1 * peak < rate <= 1.05 * peak, (kind, rate)
    with pytest.raises(H.HsvdError):
        H.debug_probe("mfma_f64", None, 0)
