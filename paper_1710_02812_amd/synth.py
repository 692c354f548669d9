"""Seeded synthetic inputs shaped like the paper's dense low-rank workloads.

The paper measures on CFD snapshot matrices and a face-image matrix (Section 4),
none of which is available here; these generators stand in for them.  The module
holds input construction only (random draws, random orthonormal bases and the
closed-form snapshot field); it contains none of the hierarchical SVD's
arithmetic, so both the CPU oracle and the GPU path can consume its arrays.

Conventions (all generators):
  * ``rng = numpy.random.default_rng(seed)`` (PCG64); draws are made in the
    order written in each function.
  * ``orth(rng, h, r)`` is the Q factor of the QR of an h x r standard normal
    matrix with its columns multiplied by sign(diag R), i.e. Haar distributed.
  * Matrices are built in float64; FP32 workloads round that array once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def orth(rng: np.random.Generator, h: int, r: int) -> np.ndarray:
    """h x r matrix with orthonormal columns, Haar distributed."""
    g = rng.standard_normal((h, r))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d


def low_rank(rng: np.random.Generator, m: int, n: int, sigma: np.ndarray,
             noise: float = 0.0) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """A = U diag(sigma) V^T + noise * N(0,1); returns (A, U, sigma, V).

    Draw order: U, V, then the noise matrix (only when noise > 0).
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    U = orth(rng, m, r)
    V = orth(rng, n, r)
    A = (U * sigma) @ V.T
    if noise > 0.0:
        A = A + noise * rng.standard_normal((m, n))
    return A, U, sigma, V


@dataclass
class Workload:
    """One synthetic problem: the matrix plus the plan parameters it is run with."""
    name: str
    A: np.ndarray                 # float64 master copy (the GPU may get a float32 rounding)
    p: int
    q: int
    k: int
    tol: float
    rule: str = "gamma"
    dtype: str = "f64"            # storage type handed to the GPU path
    meta: dict = field(default_factory=dict)


def config0(seed: int = 0) -> Workload:
    """512 x 512, rank 20 with sigma_i = 10^(-i/5) plus 1e-8 N(0,1); 2 x 2 grid, k = 20."""
    rng = np.random.default_rng(seed)
    sigma = 10.0 ** (-np.arange(20) / 5.0)
    A, U, s, V = low_rank(rng, 512, 512, sigma, noise=1e-8)
    return Workload("C0_512x512_rank20_grid2x2_k20_fp64", A, 2, 2, 20, 0.0,
                    dtype="f64", meta={"U": U, "sigma": s, "V": V})


def snapshot_matrix(rng: np.random.Generator, m: int, n: int, modes: int = 50,
                    decay: float = 8.0, noise: float = 1e-6) -> np.ndarray:
    """Snapshot-like field A[i,j] = sum_r a_r sin(pi r x_i + phi_r) cos(pi r t_j) + noise.

    x ~ U(0,1)^m, t ~ U(0,1)^n (i.i.d., unsorted), phi ~ U(0, 2 pi)^modes,
    a_r = exp(-r / decay); then noise * N(0,1) entrywise.  Draw order: x, t, phi, noise.
    """
    x = rng.uniform(0.0, 1.0, m)
    t = rng.uniform(0.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, modes)
    r = np.arange(modes, dtype=np.float64)
    a = np.exp(-r / decay)
    S = np.sin(np.pi * np.outer(x, r) + phi)          # m x modes
    C = np.cos(np.pi * np.outer(t, r))                # n x modes
    A = (S * a) @ C.T
    if noise > 0.0:
        A += noise * rng.standard_normal((m, n))
    return A


def config1(seed: int = 1, m: int = 8192, n: int = 8192, block: int = 1024) -> Workload:
    """8192 x 8192 snapshot-like matrix, 50 modes, 1e-6 noise; 8 x 8 grid of 1024^2, k = 50."""
    rng = np.random.default_rng(seed)
    A = snapshot_matrix(rng, m, n, 50, 8.0, 1e-6)
    return Workload(f"C1_snapshot_{m}x{n}_grid{m // block}x{n // block}_k50", A,
                    m // block, n // block, 50, 0.0, dtype="f32")


def config2(seed: int = 2, m: int = 16384, block: int = 1024, noise: str = "abs") -> Workload:
    """16384^2, sigma_i = exp(-i/10) (i < 256) plus Gaussian noise; 16 x 16 grid, k = 64.

    noise = "abs": 1e-5 N(0,1) entrywise (the literal reading; its spectral edge
    1e-5 * 2 sqrt(m) ~ 2.6e-3 sits at sigma_60, so the rank-64 cut falls in the noise).
    noise = "rel": 1e-5 times the signal's RMS entry, sqrt(sum sigma_i^2) / m, times
    N(0,1) (the cut then falls in the clean exp(-i/10) decay).
    """
    if noise not in ("abs", "rel"):
        raise ValueError("noise must be 'abs' or 'rel'")
    rng = np.random.default_rng(seed)
    sigma = np.exp(-np.arange(256) / 10.0)
    level = 1e-5 if noise == "abs" else 1e-5 * float(np.sqrt(np.sum(sigma ** 2))) / m
    A, U, s, V = low_rank(rng, m, m, sigma, noise=level)
    tag = "" if noise == "abs" else "_relnoise"
    return Workload(f"C2{tag}_{m}x{m}_exp10_grid{m // block}x{m // block}_k64", A,
                    m // block, m // block, 64, 0.0, dtype="f32",
                    meta={"sigma": s, "noise": level})


def config3(seed: int = 3, count: int = 200, lo: int = 256, hi: int = 4096,
            block: int = 512, rank_hi: int = 80) -> list[Workload]:
    """Uneven batch: m, n ~ U{lo..hi}, rank ~ U{5..rank_hi}, sigma_i = exp(-i/6), no noise.

    Grids p = ceil(m/block), q = ceil(n/block) (balanced split), k = rank.
    Draw order per matrix: m, n, rank, U, V.
    """
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        m = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(lo, hi + 1))
        rank = int(rng.integers(5, rank_hi + 1))
        sigma = np.exp(-np.arange(rank) / 6.0)
        A, U, s, V = low_rank(rng, m, n, sigma)
        out.append(Workload(f"C3_{j}_{m}x{n}_r{rank}", A, -(-m // block), -(-n // block),
                            rank, 0.0, dtype="f32", meta={"sigma": s}))
    return out


def config4(seed: int = 4, p: int = 32, q: int = 8, block: int = 1024,
            base_rank: int = 128, max_class: int = 5, k: int = 256) -> Workload:
    """Per-block local ranks from a smooth seeded field over shared orthonormal bases.

    phi1, phi2 ~ U(0, 2 pi); f(I,J) = 1/2 + 1/2 sin(2 pi I/p + phi1) cos(2 pi J/q + phi2);
    class c = min(max_class, floor((max_class + 1) f)); r_IJ = 4 * 2^c (max_class = 5
    gives ranks 4..128; 3 gives 4..32, whose leaf ranks fit a rank cap of 64).  Shared bases Ubar (m x 128),
    Vbar (n x 128); block (I,J) = Ubar_I diag(exp(-4 i / r_IJ)) Vbar_J^T.  Frobenius
    rule with tol = 1e-3.  Draw order: phi1, phi2, Ubar, Vbar.
    """
    rng = np.random.default_rng(seed)
    phi1, phi2 = rng.uniform(0.0, 2.0 * math.pi, 2)
    m, n = p * block, q * block
    Ub = orth(rng, m, base_rank)
    Vb = orth(rng, n, base_rank)
    I = np.arange(p)[:, None]
    J = np.arange(q)[None, :]
    f = 0.5 + 0.5 * np.sin(2 * np.pi * I / p + phi1) * np.cos(2 * np.pi * J / q + phi2)
    cls = np.minimum(max_class, np.floor((max_class + 1) * f)).astype(int)
    ranks = 4 * (2 ** cls)
    A = np.empty((m, n))
    i = np.arange(base_rank, dtype=np.float64)
    for bi in range(p):
        for bj in range(q):
            d = np.exp(-4.0 * i / ranks[bi, bj])
            A[bi * block:(bi + 1) * block, bj * block:(bj + 1) * block] = \
                (Ub[bi * block:(bi + 1) * block] * d) @ Vb[bj * block:(bj + 1) * block].T
    return Workload(f"C4_{m}x{n}_field_grid{p}x{q}", A, p, q, k, 1e-3, rule="frob",
                    dtype="f32", meta={"block_ranks": ranks})


def sketch_pair(seed: int, m: int, n: int, t: int = 32) -> tuple[np.ndarray, np.ndarray]:
    """Seeded Gaussian test matrices H (m x t) and G (n x t) for two-sided sketches.

    For any m x n matrix D, E ||H^T D G||_F^2 = t^2 ||D||_F^2, so a stored t x t sketch
    H^T X G of a reference factorisation lets the Frobenius distance of a candidate be
    estimated without keeping the reference's m x k and n x k factors.  Draw order: H, G.
    """
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((m, t))
    G = rng.standard_normal((n, t))
    return H, G
