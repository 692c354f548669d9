"""CPU float64 oracle of the hierarchical merge-and-truncate (MAT) truncated SVD.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the library's own execution path never
calls it and shares no code with it.

It follows Vasudevan & Ramakrishna, "A Hierarchical Singular Value Decomposition
Algorithm for Low Rank Matrices" (arXiv:1710.02812):

  * Section 3, Algorithm 1 (DoSVDofBlocks / DoSVDofColSlices / DoMergeOfSlices /
    BlockMerge): row slabs outermost; inside each slab the column blocks get
    truncated SVDs that are merged pairwise up a tree (left factors only); the
    slab's right factor comes from the SVD of U_i^T X_i; the slab nodes are then
    merged pairwise the same way (right factors only).
  * Section 3, truncation: keep singular values >= gamma * sigma_1 of the matrix
    being truncated, before and after every merge.
  * Section 3, left vectors by projection: SVD(X V) = U_y S_y V_y^T gives
    U = U_y, S = S_y, V = V V_y.
  * Section 3, Algorithm 2: iterative improvement (a power step on the subspace).

Each step uses the plain definition with LAPACK SVDs: a merge is the truncated
SVD of the concatenated scaled factors [U1 S1, U2 S2] (the column-split
identity of Section 3); the faster complement form (eqs. orthmerge1/orthmerge)
is implemented separately in ``merge_complement`` and is used only to cross-check
that identity, never as the reference.

Readings where the paper is silent or garbled:
  R1 truncation keeps s_i >= tol * s_0 (ties kept), caps r <= k, and drops values
     <= max(shape) * 2^-52 * s_0 (numerical zero).  tol = 0 means fixed rank k.
  R2 the same rule is applied to leaves, merges and the slab re-projection; the
     final projection applies only the zero floor.
  R3 E's lower-right block is R S2 (the printed S2 R does not follow from
     U2 S2 = U1 (U1^T U2) S2 + U_o R S2), and V = diag(V1, V2) V_E.
  R4 slice counts: the block grid is given as counts (p, q); rows/columns are
     split evenly, the first (m mod p) row blocks one row taller.
  R5 the tree pairs neighbours (0,1), (2,3), ... left to right and carries an odd
     last node up unchanged, looping until one node is left.
  R6 Algorithm 2 updates V-hat every iteration; the rank is frozen.
  R7 a rank-0 node is the identity of a merge.
  R8 singular vector signs: flip (u_i, v_i) so that the entry of u_i with the
     largest magnitude is positive (ties: lowest index).
  R9 'frob' rule (used by the learned-rank workload): smallest r whose discarded
     tail energy sum_{i>=r} s_i^2 is <= tol^2 * sum s_i^2, then the zero floor.
  R17 Algorithm 2's error is tested after every iteration, the first one included
     (against the Sigma-hat it was given, Algorithm 1's), and the loop ends at the
     first error <= eps.
  R18 the opposite order of the two sets of merges (Section 3: either order gives the
     singular values and one side's vectors) merges the blocks' right factors inside
     each column slab, re-projects U_j from SVD(X_j V_j), merges the (U_j, S_j) up the
     column-slab tree and projects V from SVD(X^T U).
  R19 Gram input (the method applied to X^T X, as in Section 4's runs that form the product
     first and then split it into blocks):
     the trees run on G = X^T X formed in float64, with the grid, tol and rule taken
     on G; V-hat from G's row-slab tree is X's, and U, s come from projecting X itself
     (not from square roots of G's values), so the results are X's factors.
"""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -52


# ----------------------------------------------------------------------------- partition
def balanced_split(n: int, parts: int) -> list[tuple[int, int]]:
    """Half-open [start, stop) ranges splitting n into `parts` nearly equal pieces (R4).

    Algorithm 1 fills its lists with row/column slices of fixed size d (or c); with
    the grid given as counts the sizes differ by at most one, larger pieces first.
    """
    if parts < 1 or parts > max(n, 1):
        raise ValueError("need 1 <= parts <= n")
    base, extra = divmod(n, parts)
    out, start = [], 0
    for i in range(parts):
        size = base + (1 if i < extra else 0)
        out.append((start, start + size))
        start += size
    return out


# ----------------------------------------------------------------------------- truncation
def truncation_rank(s, k: int, tol: float, rule: str, shape) -> int:
    """Number of leading singular values kept (Section 3 truncation criterion; R1, R9).

    `s` is sorted in decreasing order; `shape` is the shape of the matrix whose
    singular values these are (it scales the numerical-zero floor).
    """
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or not s[0] > 0.0:
        return 0
    floor = max(shape) * EPS * s[0]
    nonzero = int(np.count_nonzero(s > floor))
    if rule == "gamma":
        r = int(np.count_nonzero(s >= tol * s[0]))
    elif rule == "frob":
        e = s * s
        tail = np.concatenate([np.cumsum(e[::-1])[::-1], [0.0]])   # tail[r] = sum_{i>=r} e_i
        r = int(np.argmax(tail <= tol * tol * e.sum()))
    else:
        raise ValueError(f"unknown rule {rule!r}")
    return min(r, nonzero, k)


def _svd(M: np.ndarray):
    """Thin LAPACK SVD that also accepts matrices with an empty dimension."""
    h, w = M.shape
    if h == 0 or w == 0:
        return np.zeros((h, 0)), np.zeros(0), np.zeros((0, w))
    return np.linalg.svd(M, full_matrices=False)


# ----------------------------------------------------------------------------- one MAT step
def leaf(block: np.ndarray, k: int, tol: float, rule: str):
    """Truncated SVD of one block: Algorithm 1, DoSVDofColSlices' per-slice SVD."""
    U, s, _ = _svd(block)
    r = truncation_rank(s, k, tol, rule, block.shape)
    return U[:, :r], s[:r]


def randomised_leaf(block: np.ndarray, k: int, tol: float, rule: str, omega: np.ndarray,
                    power: int):
    """Truncated SVD of one block by a randomised range finder (Conclusions: the block
    SVDs may be randomised), used only to measure how far such leaves move the result
    from the exact ones.

    omega (cols x l) is the Gaussian test matrix, passed in.  Y = block omega; then
    `power` times Q = orth(Y), Z = orth(block^T Q), Y = block Z; Q = orth(Y);
    B = Q^T block = U_B S V^T; the leaf is (Q U_B, S) truncated by the same rule.
    """
    Q, _ = np.linalg.qr(block @ omega)
    for _ in range(power):
        Z, _ = np.linalg.qr(block.T @ Q)
        Q, _ = np.linalg.qr(block @ Z)
    Ub, s, _ = _svd(Q.T @ block)
    r = truncation_rank(s, k, tol, rule, block.shape)
    return (Q @ Ub)[:, :r], s[:r]


def merge(U1, s1, U2, s2, k: int, tol: float, rule: str):
    """One merge-and-truncate step on left factors (Section 3, column-split identity).

    [X1 X2] ~ [U1 S1, U2 S2] diag(V1^T, V2^T); the left singular vectors and values
    of [X1 X2] are those of F = [U1 S1, U2 S2], truncated by the same rule.  The
    row-split case is the same operation on right factors (F = [V1 S1, V2 S2]).
    """
    F = np.hstack([U1 * s1, U2 * s2])
    U, s, _ = _svd(F)
    r = truncation_rank(s, k, tol, rule, F.shape)
    return U[:, :r], s[:r]


def merge_complement(U1, s1, U2, s2, k: int | None = None, tol: float = 0.0,
                     rule: str = "gamma", truncate: bool = True):
    """The orthogonal-complement form of one merge (Section 3, eqs. orthmerge1/orthmerge).

    Q = U2 - U1 (U1^T U2) = U_o R;  E = [[S1, (U1^T U2) S2], [0, R S2]] (reading R3);
    E = U_E S_E V_E^T;  U = [U1 U_o] U_E, S = S_E.  Used only to cross-check the
    identity against ``merge``.  Returns (U, s, pieces) where pieces holds
    Uo, E and V_E for reconstruction checks.
    """
    C = U1.T @ U2
    Q = U2 - U1 @ C
    Uo, R = np.linalg.qr(Q)
    k1, k2 = s1.size, s2.size
    E = np.zeros((k1 + R.shape[0], k1 + k2))
    E[:k1, :k1] = np.diag(s1)
    E[:k1, k1:] = C * s2
    E[k1:, k1:] = R * s2
    UE, sE, VEt = _svd(E)
    U = np.hstack([U1, Uo]) @ UE
    r = sE.size
    if truncate:
        r = truncation_rank(sE, k if k is not None else sE.size, tol, rule,
                            (U1.shape[0], k1 + k2))
    return U[:, :r], sE[:r], {"Uo": Uo, "E": E, "VEt": VEt, "UE": UE, "sE": sE}


def merge_tree(nodes, k: int, tol: float, rule: str, merge_fn=None):
    """Pairwise merge levels until one node is left (Algorithm 1, DoMergeOfSlices; R5, R7)."""
    merge_fn = merge if merge_fn is None else merge_fn
    nodes = list(nodes)
    if not nodes:
        raise ValueError("empty node list")
    while len(nodes) > 1:
        nxt = [merge_fn(*nodes[i], *nodes[i + 1], k, tol, rule)
               for i in range(0, len(nodes) - 1, 2)]
        if len(nodes) % 2:
            nxt.append(nodes[-1])
        nodes = nxt
    return nodes[0]


# ----------------------------------------------------------------------------- Algorithm 1
def slab_nodes(A, p: int, q: int, k: int, tol: float, rule: str, merge_fn=None, leaf_fn=None):
    """For each row slab: column MAT tree, then V_i, S_i = SVD(U_i^T X_i) (Algorithm 1).

    leaf_fn(block, k, tol, rule, i, j) replaces the exact leaf SVD of block (i, j)."""
    m, n = A.shape
    out = []
    for i, (r0, r1) in enumerate(balanced_split(m, p)):
        X = A[r0:r1]
        if leaf_fn is None:
            leaves = [leaf(X[:, c0:c1], k, tol, rule) for (c0, c1) in balanced_split(n, q)]
        else:
            leaves = [leaf_fn(X[:, c0:c1], k, tol, rule, i, j)
                      for j, (c0, c1) in enumerate(balanced_split(n, q))]
        Ui, si = merge_tree(leaves, k, tol, rule, merge_fn)
        W = Ui.T @ X                                    # r_i x n
        _, sw, Vwt = _svd(W)
        r = truncation_rank(sw, k, tol, rule, W.shape)  # R2
        out.append((Vwt[:r].T, sw[:r]))
    return out


def col_slab_nodes(A, p: int, q: int, k: int, tol: float, rule: str, merge_fn=None):
    """The opposite order of the two sets of merges (Section 3): for each column slab
    X_j, the blocks' right factors (V_b, S_b) -- the left factors of X_b^T -- are merged
    pairwise up a tree (the row-wise merge of S_b V_b^T), then U_j, S_j = SVD(X_j V_j)
    truncated by the same rule (R2).  Returns the column-slab nodes (U_j, S_j)."""
    m, n = A.shape
    out = []
    for (c0, c1) in balanced_split(n, q):
        X = A[:, c0:c1]
        leaves = [leaf(X[r0:r1].T, k, tol, rule) for (r0, r1) in balanced_split(m, p)]
        Vj, _ = merge_tree(leaves, k, tol, rule, merge_fn)
        Y = X @ Vj                                       # m x r_j
        Uy, sy, _ = _svd(Y)
        r = truncation_rank(sy, k, tol, rule, Y.shape)
        out.append((Uy[:, :r], sy[:r]))
    return out


def project(A, V):
    """Left vectors by projection: SVD(A V) = U_y S_y V_y^T; U = U_y, V <- V V_y (Section 3)."""
    Y = A @ V
    Uy, sy, Vyt = _svd(Y)
    r = truncation_rank(sy, sy.size, 0.0, "gamma", Y.shape)   # zero floor only (R2)
    return Uy[:, :r], sy[:r], V @ Vyt[:r].T


def improve(A, V, s_hat, iters: int, eps: float | None = None):
    """Algorithm 2 (iterative improvement; R6, R17).

    Input: A, V-hat (n x r) and Sigma-hat (r values: Algorithm 1's singular values).
    Each iteration: U_i = left singular vectors of A V-hat (r of them);
    U~ S~ V~^T = SVD(U_i^T A); Error = ||Sigma-hat - S~||_2 / ||Sigma-hat||_2;
    Sigma-hat <- S~, V-hat <- V~, U-hat = U_i U~.  The loop is a do-while: the first
    iteration is tested against the input Sigma-hat, and the loop ends at the first
    Error <= eps (eps None: exactly `iters` iterations; otherwise at most `iters`).
    Returns (U-hat, Sigma-hat, V-hat, iterations run).
    """
    s_hat = np.asarray(s_hat, dtype=np.float64)
    r = V.shape[1]
    U = None
    t = 0
    for t in range(1, iters + 1):
        Ui, _, _ = _svd(A @ V)
        Ui = Ui[:, :r]
        Ut, st, Vtt = _svd(Ui.T @ A)
        U, V = Ui @ Ut, Vtt.T
        den = np.linalg.norm(s_hat)
        err = np.linalg.norm(s_hat - st) / den if den > 0.0 else 0.0
        s_hat = st
        if eps is not None and err <= eps:
            break
    return U, s_hat, V, t


def sign_normalise(U, V):
    """Flip (u_i, v_i) so the largest-magnitude entry of u_i is positive (R8)."""
    U = U.copy()
    V = V.copy()
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        if U[j, i] < 0.0:
            U[:, i] *= -1.0
            V[:, i] *= -1.0
    return U, V


def hsvd(A, p: int, q: int, k: int, tol: float = 0.0, rule: str = "gamma",
         refine: int = 0, merge_fn=None, refine_eps: float | None = None, leaf_fn=None,
         info: dict | None = None, order: str = "rows_last"):
    """The whole method: returns (U [m x k], s [k], Vt [k x n], r), zero padded past r.

    order "rows_last" (Algorithm 1 as printed): the row-slab tree gives (V-hat, S-hat)
    and U follows by projection.  order "cols_last" (the opposite order of the two sets
    of merges, Section 3): the column-slab tree of `col_slab_nodes` gives (U-hat, S-hat)
    and V follows by the projection SVD(A^T U-hat).  `refine` runs that many iterations
    of Algorithm 2 (fewer when refine_eps stops them, as in `improve`, whose input
    Sigma-hat is the tree's); for cols_last they are Algorithm 2 stated for A^T, whose
    right vectors are A's left ones.  `info`, when given, receives the iterations of
    Algorithm 2 actually run.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= p <= m and 1 <= q <= n and 1 <= k <= min(m, n) and 0.0 <= tol < 1.0):
        raise ValueError("invalid arguments")
    if order not in ("rows_last", "cols_last"):
        raise ValueError("order must be rows_last or cols_last")
    if order == "rows_last":
        slabs = slab_nodes(A, p, q, k, tol, rule, merge_fn, leaf_fn)
        Vh, sh = merge_tree(slabs, k, tol, rule, merge_fn)
        U, s, V = project(A, Vh)
    else:
        if leaf_fn is not None:
            raise ValueError("leaf_fn applies to rows_last")
        slabs = col_slab_nodes(A, p, q, k, tol, rule, merge_fn)
        Uh, sh = merge_tree(slabs, k, tol, rule, merge_fn)
        V, s, U = project(A.T, Uh)                       # A^T U-hat = V_y S_y W^T, U = U-hat W
    r = s.size
    done = 0
    if refine > 0 and r > 0:
        if order == "rows_last":
            U, s, V, done = improve(A, V, sh[:r], refine, refine_eps)
        else:
            V, s, U, done = improve(A.T, U, sh[:r], refine, refine_eps)
    if info is not None:
        info["refine_iterations"] = done
    U, V = sign_normalise(U, V)
    Uo = np.zeros((m, k))
    so = np.zeros(k)
    Vto = np.zeros((k, n))
    Uo[:, :r] = U
    so[:r] = s
    Vto[:r] = V.T
    return Uo, so, Vto, r


def hsvd_gram(X, p: int, q: int, k: int, tol: float = 0.0, rule: str = "gamma",
              refine: int = 0, refine_eps: float | None = None, info: dict | None = None):
    """The method applied to the Gram matrix G = X^T X (R19), returning X's factors.

    G's right singular vectors are X's and its singular values are X's squared, so
    Algorithm 1's row-slab tree runs on G (p x q grid over n x n; `tol` and `rule`
    apply to G's values), V-hat is taken from its root and U, s follow by the projection
    SVD(X V-hat) of Section 3.  Algorithm 2 runs on X; its first iteration is tested
    against the projection's singular values.  Returns (U, s, Vt, r) as `hsvd`.
    """
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    if not (1 <= p <= n and 1 <= q <= n and 1 <= k <= min(m, n) and 0.0 <= tol < 1.0):
        raise ValueError("invalid arguments")
    G = X.T @ X
    slabs = slab_nodes(G, p, q, k, tol, rule)
    Vh, _ = merge_tree(slabs, k, tol, rule)
    U, s, V = project(X, Vh)
    r = s.size
    done = 0
    if refine > 0 and r > 0:
        U, s, V, done = improve(X, V, s, refine, refine_eps)
    if info is not None:
        info["refine_iterations"] = done
    U, V = sign_normalise(U, V)
    Uo = np.zeros((m, k))
    so = np.zeros(k)
    Vto = np.zeros((k, n))
    Uo[:, :r] = U
    so[:r] = s
    Vto[:r] = V.T
    return Uo, so, Vto, r


def flop_model(m: int, n: int, P: int, k: int) -> dict:
    """Section 3.1 cost model for a column split into P blocks of s = n/P columns."""
    s = n / P
    return {
        "full_svd": 6 * m * n * n + 16 * n ** 3,
        "blocks": P * (6 * m * s * s + 16 * s ** 3),
        "merges": (P - 1) * (14 * m * k * k + 176 * k ** 3),
        "bound": 20 * m * n * n / P + 192 * n ** 3 / P ** 2,
    }
