"""Reference values and intrinsic accuracy floor of the 16384^2 mixed-precision workload,
from the oracle alone.

Writes tests/golden/c2_reference.json (--what reference) and tests/golden/c2_floor.json
(--what floor).  Calls only oracle/ and the input generator.

Reference: the oracle's rank, its k singular values, its residual ‖A - X_o‖_F / ‖A‖_F
and a two-sided sketch H^T X_o G (64 x 64, H and G from synth.sketch_pair with seed
2002), X_o = U_o diag(s_o) V_o^T.  A candidate's Frobenius distance to X_o is then
estimated as ‖H^T X G - H^T X_o G‖_F / 64 (unbiased in the square; relative standard
deviation about 5 % for differences of rank ~100), without the reference's factors.

The workload: A = U diag(s) V^T + 1e-5 N(0,1), s_i = exp(-i/10) for i < 256, rounded
to float32; 16 x 16 grid of 1024^2 blocks, k = 64, tol = 0.  Its rank-64 cut falls where
the noise edge meets the signal, so two results that are each correct can still differ.
The floors bound how close any implementation can come to the exact-leaf oracle:

  F1 = e_F(oracle(A32), oracle(bf16(A32)))    -- rounding the input to bfloat16 alone
  F2 = e_F(oracle(A32), oracle with randomised leaves, l = 80, one power step)
       -- the leaf mechanism alone (Conclusions: randomised block SVDs)

Also recorded: the rank r* of the leading well-separated modes (largest r with
s_r / s_{r+1} >= 1.05 in the oracle) with e_F restricted to those modes, and the
residual difference |‖A - X1‖_F - ‖A - X2‖_F| / ‖A‖_F, which ignores rotations inside
near-degenerate modes.

The same for the relative-noise reading (--noise rel: noise 1e-5 times the signal's RMS
entry, so the cut falls in the clean exp(-i/10) decay), written to c2_relnoise_*.json.

Usage: python tests/golden/make_c2_floor.py --what reference|floor [--noise abs|rel] [--size 16384]
(about 3 minutes for the reference and 8 for the floor on 8 cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import metrics  # noqa: E402
from paper_1710_02812_amd import synth  # noqa: E402


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def residual(A, U, s, Vt, r):
    """‖A - U diag(s) Vt‖_F by the energy identity (U, Vt orthonormal projections)."""
    # ‖A - U S V^T‖^2 = ‖A‖^2 - 2 tr(S U^T A V) + ‖S‖^2
    Ur, sr, Vr = U[:, :r], s[:r], Vt[:r].T
    cross = np.einsum("i,i->", sr, np.einsum("ij,ij->j", Ur, A @ Vr))
    return float(np.sqrt(max(np.sum(A * A) - 2.0 * cross + np.sum(sr * sr), 0.0)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=16384)
    ap.add_argument("--what", choices=["reference", "floor"], default="floor")
    ap.add_argument("--noise", choices=["abs", "rel"], default="abs",
                    help="abs: 1e-5 N(0,1) (the literal reading); rel: 1e-5 x the signal's RMS entry")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    here = os.path.dirname(os.path.abspath(__file__))
    if args.out is None:
        tag = "" if args.noise == "abs" else "_relnoise"
        args.out = os.path.join(here, f"c2{tag}_{args.what}.json")
    w = synth.config2(2, m=args.size, noise=args.noise)
    A32 = w.A.astype(np.float32).astype(np.float64)
    del w.A
    out = {"workload": w.name, "m": args.size, "n": args.size, "p": w.p, "q": w.q, "k": w.k,
           "tol": w.tol, "seed": 2, "noise": w.meta["noise"],
           "input": "float32 rounding of the float64 generator output"}
    t0 = time.time()
    ref = oracle.hsvd(A32, w.p, w.q, w.k, w.tol)
    print(f"exact-leaf oracle {time.time() - t0:.1f} s", flush=True)
    U0, s0, Vt0, r0 = ref
    out["rank"] = int(r0)
    if args.what == "reference":
        nA = float(np.sqrt(np.sum(A32 * A32)))
        H, G = synth.sketch_pair(2002, A32.shape[0], A32.shape[1], 64)
        sk = (H.T @ (U0[:, :r0] * s0[:r0])) @ (Vt0[:r0] @ G)
        out["sigma"] = [float(x) for x in s0[:r0]]
        out["rel_residual"] = residual(A32, U0, s0, Vt0, r0) / nA
        out["sketch_seed"] = 2002
        out["sketch_t"] = 64
        out["sketch"] = [[float(x) for x in row] for row in sk]
        with open(args.out, "w") as f:
            json.dump(out, f)
        print({kk: v for kk, v in out.items() if kk != "sketch"})
        return

    t0 = time.time()
    Ab = bf16_round(A32)
    bf = oracle.hsvd(Ab, w.p, w.q, w.k, w.tol)
    del Ab
    print(f"bf16-input oracle {time.time() - t0:.1f} s", flush=True)
    c1 = metrics.compare(*bf, *ref)
    out["F1"] = c1

    rng = np.random.default_rng(1002)
    bs = args.size // w.q
    omegas = {}

    def rleaf(block, k, tol, rule, i, j):
        key = (i, j)
        if key not in omegas:
            omegas[key] = rng.standard_normal((block.shape[1], 80))
        return oracle.randomised_leaf(block, k, tol, rule, omegas.pop(key), 1)

    t0 = time.time()
    rl = oracle.hsvd(A32, w.p, w.q, w.k, w.tol, leaf_fn=rleaf)
    print(f"randomised-leaf oracle {time.time() - t0:.1f} s", flush=True)
    out["F2"] = metrics.compare(*rl, *ref)

    s = s0[:r0]
    ratios = s[:-1] / s[1:]
    sep = [i + 1 for i in range(ratios.size) if ratios[i] >= 1.05]
    rstar = max(sep) if sep else 0
    out["r_star"] = int(rstar)
    for name, cand in (("F1", bf), ("F2", rl)):
        U, sc, Vt, _ = cand
        if rstar > 0:
            out[name]["e_frob_leading"] = metrics.e_frob(U[:, :rstar], sc[:rstar], Vt[:rstar].T,
                                                         U0[:, :rstar], s0[:rstar], Vt0[:rstar].T)
        nA = float(np.sqrt(np.sum(A32 * A32)))
        out[name]["residual_diff"] = abs(residual(A32, U, sc, Vt, r0) -
                                         residual(A32, U0, s0, Vt0, r0)) / nA
    out["oracle_sigma_near_cut"] = [float(x) for x in s0[max(0, r0 - 4):r0]]
    out["floor"] = max(out["F1"]["e_frob"], out["F2"]["e_frob"])
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
