"""End-to-end parity of the HIP path (hsvd_execute through the C ABI) against the
CPU float64 oracle on the same seeded inputs.

Gates (float64 path): e_sigma <= 1e-10, e_frob <= 1e-10 and, where the oracle's
subspace amplification sigma_1/(sigma_r - sigma_{r+1}) is <= 1e4, the principal
angle sines <= max(1e-10, 10 * 2^-52 * amplification): two backward-stable
computations of a subspace differ by O(eps * amplification), which stays below
1e-10 for every amplification up to 1e4 -- the gate is 1e-10 wherever it applies.
The float32-storage path is gated at e_frob <= 1e-5.  Integer outputs (the rank)
are compared exactly.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import metrics  # noqa: E402
from paper_1710_02812_amd import hsvd as H, synth  # noqa: E402

DEV = "cuda:0"


def run_gpu(A, p, q, k, tol=0.0, dtype=torch.float64, **opts):
    At = torch.tensor(A, dtype=dtype, device=DEV)
    U, S, Vt, r = H.svd(At, p, q, k, tol, **opts)
    torch.cuda.synchronize()
    return U.double().cpu().numpy(), S.double().cpu().numpy(), Vt.double().cpu().numpy(), r


def oracle_order(m, n, opts):
    """The merge order a plan takes: HSVD_ORDER_AUTO runs the opposite order (column
    slabs merged last) for a short-fat matrix, Algorithm 1's otherwise."""
    order = opts.get("order", H.ORDER_AUTO)
    if order == H.ORDER_COLS_LAST or (order == H.ORDER_AUTO and m < n):
        return "cols_last"
    return "rows_last"


def check_parity(A, p, q, k, tol=0.0, rule="gamma", dtype=torch.float64, gate=1e-10, **opts):
    Ao = A if dtype == torch.float64 else A.astype(np.float32).astype(np.float64)
    Uo, so, Vto, ro = oracle.hsvd(Ao, p, q, k, tol, rule, order=oracle_order(*A.shape, opts))
    Ug, sg, Vtg, rg = run_gpu(A, p, q, k, tol, dtype,
                              rule=(H.RULE_GAMMA if rule == "gamma" else H.RULE_FROB), **opts)
    assert rg == ro, (rg, ro)
    c = metrics.compare(Ug, sg, Vtg, rg, Uo, so, Vto, ro)
    print(c, flush=True)
    assert c["e_sigma"] <= gate
    assert c["e_frob"] <= gate
    # zero padding past the rank
    assert np.all(sg[rg:] == 0) and np.all(Ug[:, rg:] == 0) and np.all(Vtg[rg:] == 0)
    # sign convention: largest-magnitude entry of each u_i positive
    for i in range(rg):
        j = np.argmax(np.abs(Ug[:, i]))
        assert Ug[j, i] > 0
    if ro > 0 and dtype == torch.float64:
        s_full = np.linalg.svd(Ao, compute_uv=False) if Ao.size <= 4e6 else None
        if s_full is not None:
            amp = metrics.amplification(s_full, ro)
            if amp <= 1e4:
                tol_sin = max(1e-10, 10.0 * 2.0 ** -52 * amp)
                assert c["sin_u"] <= tol_sin and c["sin_v"] <= tol_sin, (c, amp)
    return c


def test_config0_fp64_parity():
    """C0: 512^2, rank 20 + 1e-8 noise, 2 x 2 grid, k = 20 (the small configuration)."""
    w = synth.config0(0)
    print("C0", flush=True)
    check_parity(w.A, w.p, w.q, w.k, w.tol)


def test_config0_fp64_fixed_power_step_count():
    """power_steps = 3 given explicitly (no convergence test) also meets the gates on C0.
    The leaf gap at the cut is ~250 (signal s_19 / 2 against a noise edge ~3e-7), so the
    subspace-iteration bound (1/250)^(2t+1) times the test matrix's factor (10..1000) is
    ~1e-10 after two steps (measured: sin_v 1.1e-10) and ~1e-15 after three."""
    w = synth.config0(0)
    check_parity(w.A, w.p, w.q, w.k, w.tol, power_steps=3)


def test_config1_fp64_parity():
    """The 8192^2 snapshot-like workload (50 modes + 1e-6 noise, 8 x 8 grid, k = 50) on
    the float64 path: e_sigma, e_frob and both principal-angle sines <= 1e-10.  The
    amplification is bounded with the noise edge 1e-6 (sqrt m + sqrt n) >= s_51."""
    w = synth.config1(1)
    print("C1 fp64: oracle", flush=True)
    Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, w.tol)
    print("C1 fp64: GPU", flush=True)
    Ug, sg, Vtg, rg = run_gpu(w.A, w.p, w.q, w.k, w.tol)
    assert rg == ro == 50
    c = metrics.compare(Ug, sg, Vtg, rg, Uo, so, Vto, ro)
    print(c, flush=True)
    edge = 1e-6 * (np.sqrt(w.A.shape[0]) + np.sqrt(w.A.shape[1]))
    amp = so[0] / (so[ro - 1] - edge)
    assert amp <= 1e4
    for key in ("e_sigma", "e_frob", "sin_u", "sin_v"):
        assert c[key] <= 1e-10, (key, c)


@pytest.mark.parametrize("seed", [100, 101])
def test_config0_other_seeds(seed):
    w = synth.config0(seed)
    check_parity(w.A, w.p, w.q, w.k, w.tol)


@pytest.mark.parametrize("m,n,p,q,k", [(1000, 900, 3, 4, 20), (700, 1300, 5, 3, 12),
                                       (513, 257, 2, 1, 9), (257, 513, 1, 3, 9),
                                       (640, 640, 5, 5, 30)])
def test_ragged_grids_fp64(m, n, p, q, k):
    """Ragged blocks (balanced split), odd carries, both tree directions."""
    rng = np.random.default_rng(m + n + p + q)
    sigma = 10.0 ** (-np.arange(k) / (k / 3.0))
    A, *_ = synth.low_rank(rng, m, n, sigma, noise=1e-9)
    print(f"ragged {m}x{n} {p}x{q} k={k}", flush=True)
    check_parity(A, p, q, k)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 3), (8, 8), (3, 5)])
def test_exact_low_rank_recovery(p, q):
    """rank(A) < k: rank found exactly and the constructed factors recovered."""
    rng = np.random.default_rng(7 * p + q)
    A, U0, s0, V0 = synth.low_rank(rng, 800, 600, np.array([4.0, 2.0, 1.0, 0.5, 0.25]))
    U, s, Vt, r = run_gpu(A, p, q, 12)
    assert r == 5
    assert metrics.e_sigma(s[:r], s0) <= 1e-12
    assert metrics.e_frob(U[:, :r], s[:r], Vt[:r].T, U0, s0, V0) <= 1e-12


def test_zero_matrix():
    A = np.zeros((300, 200))
    U, s, Vt, r = run_gpu(A, 2, 2, 5)
    assert r == 0 and np.all(s == 0) and np.all(U == 0) and np.all(Vt == 0)


def test_gamma_rule_with_tol():
    """tol > 0: the gamma rule cuts inside the spectrum (gap at the cut)."""
    rng = np.random.default_rng(3)
    sigma = np.concatenate([np.linspace(10, 2, 8), np.linspace(0.05, 0.01, 10)])
    A, *_ = synth.low_rank(rng, 600, 500, sigma, noise=1e-10)
    c = check_parity(A, 3, 2, 20, tol=0.1)
    assert c["rank"] == 8


def test_frob_rule():
    rng = np.random.default_rng(4)
    sigma = np.concatenate([np.linspace(10, 5, 6), 1e-3 * np.ones(6)])
    A, *_ = synth.low_rank(rng, 512, 384, sigma, noise=1e-12)
    c = check_parity(A, 2, 2, 16, tol=1e-2, rule="frob")
    assert c["rank"] == 6


def test_fp32_storage_small():
    w = synth.config0(0)
    check_parity(w.A, w.p, w.q, w.k, w.tol, dtype=torch.float32, gate=1e-5)


def test_refinement_step_matches_oracle():
    """One Algorithm 2 iteration after the projection (refine_steps = 1)."""
    rng = np.random.default_rng(9)
    sigma = np.exp(-np.arange(30) / 4.0)
    A, *_ = synth.low_rank(rng, 600, 600, sigma, noise=1e-9)
    Uo, so, Vto, ro = oracle.hsvd(A, 3, 3, 20, 0.0, "gamma", refine=1)
    Ug, sg, Vtg, rg = run_gpu(A, 3, 3, 20, refine_steps=1)
    assert rg == ro
    c = metrics.compare(Ug, sg, Vtg, rg, Uo, so, Vto, ro)
    print(c)
    assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10


def _refine_case():
    rng = np.random.default_rng(9)
    sigma = np.exp(-np.arange(30) / 4.0)
    A, *_ = synth.low_rank(rng, 600, 600, sigma, noise=1e-9)
    return A


def _refine_changes(A, p, k):
    """Relative changes of the singular values over Algorithm 2's iterations: entry 0
    from Algorithm 1's values (the root of the row-slab tree) to iteration 1's, entry t
    from iteration t's to iteration t + 1's."""
    slabs = oracle.slab_nodes(A, p, p, k, 0.0, "gamma")
    _, sh = oracle.merge_tree(slabs, k, 0.0, "gamma")
    ss = [oracle.hsvd(A, p, p, k, 0.0, "gamma", refine=t)[1] for t in range(1, 7)]
    ss = [sh] + [x[:sh.size] for x in ss]
    return [np.linalg.norm(ss[t] - ss[t - 1]) / np.linalg.norm(ss[t - 1]) for t in range(1, 7)]


@pytest.mark.parametrize("eps_kind", ["between", "loose", "first", "tight"])
def test_refinement_to_tolerance_matches_oracle(eps_kind):
    """Algorithm 2 iterated until the singular values change by at most eps (relative,
    2-norm), the first iteration tested against Algorithm 1's values, at most 6: the GPU
    stops at the oracle's iteration and returns its factors.  eps sits a factor of ~3
    away from the changes on either side (they fall ~8x per iteration here), far
    outside both paths' rounding."""
    A = _refine_case()
    ch = _refine_changes(A, 3, 20)
    assert all(b < a / 3 for a, b in zip(ch[1:], ch[2:])), ch
    assert ch[0] > 3 * ch[1], ch
    eps, want = {"between": (np.sqrt(ch[2] * ch[3]), 4), "loose": (1.0, 1),
                 "first": (np.sqrt(ch[0] * ch[1]), 2), "tight": (1e-300, 6)}[eps_kind]
    info = {}
    Uo, so, Vto, ro = oracle.hsvd(A, 3, 3, 20, 0.0, "gamma", refine=6, refine_eps=eps, info=info)
    assert info["refine_iterations"] == want
    At = torch.tensor(A, device=DEV)
    plan = H.Plan(600, 600, 3, 3, 20, refine_steps=6, refine_eps=eps)
    U = torch.empty((600, 20), dtype=torch.float64, device=DEV)
    S = torch.empty((20,), dtype=torch.float64, device=DEV)
    Vt = torch.empty((20, 600), dtype=torch.float64, device=DEV)
    for _ in range(2):                      # a second execute of the plan decides afresh
        print("refine_eps", eps_kind, eps, flush=True)
        plan.execute(At, U, S, Vt)
        torch.cuda.synchronize()
        assert plan.refine_iterations() == want
        rg = plan.rank()
        assert rg == ro
        c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), rg, Uo, so, Vto, ro)
        print(c, flush=True)
        assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10
    assert plan.status() & 0xFFFF == 0
    with pytest.raises(H.HsvdError):
        H._check(H.lib().hsvd_set_profiling(plan._h, 1))
    plan.close()


def test_refinement_to_tolerance_batched_waits_for_every_matrix():
    """A batch stops when every matrix meets eps: the slow matrix sets the count (4 here)
    and the fast one (exact rank, converged at once) runs as many iterations."""
    A1 = _refine_case()
    rng = np.random.default_rng(10)
    A2, *_ = synth.low_rank(rng, 400, 300, np.linspace(5.0, 1.0, 10))
    ch = _refine_changes(A1, 3, 20)
    eps = np.sqrt(ch[2] * ch[3])
    print("batched refine_eps", eps, flush=True)
    shapes = [(600, 600, 3, 3, 20), (400, 300, 2, 2, 10)]
    plan = H.BatchPlan(shapes, refine_steps=6, refine_eps=eps)
    As = [torch.tensor(A1, device=DEV), torch.tensor(A2, device=DEV)]
    Us = [torch.empty((m, k), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
    Ss = [torch.empty((k,), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
    Vts = [torch.empty((k, n), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
    plan.execute(As, Us, Ss, Vts)
    torch.cuda.synchronize()
    assert plan.refine_iterations() == 4
    rs = plan.ranks()
    assert plan.status() & 0xFFFF == 0
    plan.close()
    outs = list(zip(Us, Ss, Vts, rs))
    for (U, S, Vt, r), (A, p, k) in zip(outs, ((A1, 3, 20), (A2, 2, 10))):
        Uo, so, Vto, ro = oracle.hsvd(A, p, p, k, 0.0, "gamma", refine=4)
        assert r == ro
        c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), r, Uo, so, Vto, ro)
        print(c, flush=True)
        assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10


def test_refinement_without_tolerance_runs_every_iteration():
    """refine_eps = 0 (default): all refine_steps iterations, as before."""
    A = _refine_case()
    At = torch.tensor(A, device=DEV)
    plan = H.Plan(600, 600, 3, 3, 20, refine_steps=3)
    U = torch.empty((600, 20), dtype=torch.float64, device=DEV)
    S = torch.empty((20,), dtype=torch.float64, device=DEV)
    Vt = torch.empty((20, 600), dtype=torch.float64, device=DEV)
    plan.execute(At, U, S, Vt)
    torch.cuda.synchronize()
    assert plan.refine_iterations() == 3
    Uo, so, Vto, ro = oracle.hsvd(A, 3, 3, 20, 0.0, "gamma", refine=3)
    c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), plan.rank(), Uo, so, Vto, ro)
    assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10
    plan.close()


def test_plan_reuse_and_repeatability():
    """Two executes of one plan give bit-identical results (no stale state)."""
    w = synth.config0(0)
    At = torch.tensor(w.A, device=DEV)
    plan = H.Plan(512, 512, 2, 2, 20)
    outs = []
    for _ in range(2):
        U = torch.empty((512, 20), dtype=torch.float64, device=DEV)
        S = torch.empty((20,), dtype=torch.float64, device=DEV)
        Vt = torch.empty((20, 512), dtype=torch.float64, device=DEV)
        plan.execute(At, U, S, Vt)
        torch.cuda.synchronize()
        outs.append((U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy()))
    assert plan.status() & 0xFFFF == 0 and plan.rank() == 20
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    plan.close()


@pytest.mark.parametrize("seed", [0, 100])
def test_mixed_bf16_config0(seed):
    """Mixed path (bfloat16 matrix-core passes + float32-accurate projection and
    refinement) against the oracle on the same float32 input: e_frob <= 1e-3."""
    w = synth.config0(seed)
    A32 = w.A.astype(np.float32)
    Ao = A32.astype(np.float64)
    Uo, so, Vto, ro = oracle.hsvd(Ao, w.p, w.q, w.k, w.tol)
    At = torch.tensor(A32, device=DEV)
    U, S, Vt, r = H.svd(At, w.p, w.q, w.k, w.tol, mixed=True)
    torch.cuda.synchronize()
    c = metrics.compare(U.double().cpu().numpy(), S.double().cpu().numpy(), Vt.double().cpu().numpy(), r,
                        Uo, so, Vto, ro)
    print("mixed C0", c, flush=True)
    assert r == ro
    assert c["e_frob"] <= 1e-3 and c["e_sigma"] <= 1e-3


def test_mixed_bf16_snapshot_2048():
    """Mixed path on a 2048^2 snapshot-like matrix (4 x 4 grid of 512^2, k = 50)."""
    w = synth.config1(1, m=2048, n=2048, block=512)
    A32 = w.A.astype(np.float32)
    Uo, so, Vto, ro = oracle.hsvd(A32.astype(np.float64), w.p, w.q, w.k, 0.0)
    U, S, Vt, r = H.svd(torch.tensor(A32, device=DEV), w.p, w.q, w.k, 0.0, mixed=True)
    torch.cuda.synchronize()
    c = metrics.compare(U.double().cpu().numpy(), S.double().cpu().numpy(), Vt.double().cpu().numpy(), r,
                        Uo, so, Vto, ro)
    print("mixed 2048", c, flush=True)
    assert r == ro
    assert c["e_frob"] <= 1e-3 and c["e_sigma"] <= 1e-3


def _uneven(count, hi, rank_hi, seed=3):
    return synth.config3(seed=seed, count=count, lo=256, hi=hi, rank_hi=rank_hi)


def test_batched_uneven_fp64():
    """One batched plan over uneven matrices (exact low rank): every matrix matches
    the oracle at the float64 gate and recovers its rank."""
    ws = _uneven(12, 1300, 40)
    print("batched fp64", [w.A.shape for w in ws], flush=True)
    As = [torch.tensor(w.A, device=DEV) for w in ws]
    outs = H.svd_batched(As, [w.p for w in ws], [w.q for w in ws], [w.k for w in ws])
    torch.cuda.synchronize()
    for w, (U, S, Vt, r) in zip(ws, outs):
        Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, 0.0)
        assert r == ro == w.k
        c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), r, Uo, so, Vto, ro)
        assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10, (w.name, c)
        assert np.max(np.abs(S.cpu().numpy()[:r] - w.meta["sigma"])) <= 1e-12


@pytest.mark.parametrize("m,n,p,q,k,rank,tol", [
    (1200, 1100, 3, 3, 80, 80, 0.0),      # every merge core 160 columns
    (1000, 1300, 2, 3, 72, 72, 0.0),      # 144 columns; short-fat: column slabs merged last
    (900, 900, 3, 2, 80, 30, 1e-10),      # wide-routed merges with 60 active columns
])
def test_wide_merge_cores_fp64(m, n, p, q, k, rank, tol):
    """Rank caps above 64: merge cores of 2k > 128 columns run on the wide cores (their
    columns in a global scratch panel); float64 parity with the oracle at the 1e-10 gates."""
    rng = np.random.default_rng(m + k + rank)
    sigma = 10.0 ** (-np.arange(rank) / (rank / 3.0))
    A, *_ = synth.low_rank(rng, m, n, sigma, noise=1e-13 if tol > 0 else 1e-9)
    print(f"wide merges {m}x{n} {p}x{q} k={k} rank={rank}", flush=True)
    check_parity(A, p, q, k, tol)


def test_wide_merge_cores_mixed():
    """The mixed path with k = 80 (wide merge cores, float32 and bfloat16 passes) against
    the oracle on the float32-rounded input, at the mixed gate 1e-3."""
    rng = np.random.default_rng(80)
    sigma = np.exp(-np.arange(80) / 10.0)
    A, *_ = synth.low_rank(rng, 2048, 2048, sigma, noise=1e-7)
    print("wide merges mixed 2048", flush=True)
    check_parity(A, 4, 4, 80, 0.0, dtype=torch.float32, gate=1e-3, mixed=True)


def test_batched_uneven_wide_fp64():
    """A batch whose rank caps straddle 64 (ranks up to 80, a 1 x 1 grid among them):
    merge cores of both kinds in the same levels; every matrix matches the oracle at
    the float64 gate and recovers its rank."""
    ws = _uneven(6, 1400, 80, seed=22)
    assert max(w.k for w in ws) > 64 and min(w.k for w in ws) <= 64
    print("batched wide fp64", [(w.A.shape, w.k) for w in ws], flush=True)
    As = [torch.tensor(w.A, device=DEV) for w in ws]
    outs = H.svd_batched(As, [w.p for w in ws], [w.q for w in ws], [w.k for w in ws])
    torch.cuda.synchronize()
    for w, (U, S, Vt, r) in zip(ws, outs):
        Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, 0.0)
        assert r == ro == w.k
        c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), r, Uo, so, Vto, ro)
        assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10, (w.name, c)
        assert np.max(np.abs(S.cpu().numpy()[:r] - w.meta["sigma"])) <= 1e-12


def test_batched_wide_tall_panels_take_the_panel_qr():
    """A batch of 132 matrices of rank caps 65..72 (panels wider than the Cholesky QR's
    64 columns, and enough of them for the one-launch panel QR in the re-projection,
    projection and Algorithm 2 steps): every matrix matches the oracle at the float64
    gate and recovers its rank; float32 storage and the mixed path at their gates."""
    rng = np.random.default_rng(132)
    ws = []
    for j in range(132):
        m, n = int(rng.integers(200, 321)), int(rng.integers(200, 321))
        k = int(rng.integers(65, 73))
        A, *_ = synth.low_rank(rng, m, n, np.exp(-np.arange(k) / 8.0), noise=0.0)
        ws.append((A, k))
    shapes = [(A.shape[0], A.shape[1], 1, 1, k) for A, k in ws]
    print("batched wide tall panels", len(ws), flush=True)
    for dt, gate, opts in ((torch.float64, 1e-10, {}), (torch.float32, 1e-5, {"refine_steps": 1}),
                           (torch.float32, 1e-3, {"mixed": True})):
        As = [torch.tensor(A, dtype=dt, device=DEV) for A, _ in ws]
        outs = H.svd_batched(As, [1] * len(ws), [1] * len(ws), [k for _, k in ws], **opts)
        torch.cuda.synchronize()
        for (A, k), (U, S, Vt, r) in zip(ws[::11], outs[::11]):
            Ao = A if dt == torch.float64 else A.astype(np.float32).astype(np.float64)
            Uo, so, Vto, ro = oracle.hsvd(Ao, 1, 1, k, 0.0, refine=opts.get("refine_steps", 0))
            assert r == ro == k
            c = metrics.compare(U.double().cpu().numpy(), S.double().cpu().numpy(),
                                Vt.double().cpu().numpy(), r, Uo, so, Vto, ro)
            assert c["e_sigma"] <= gate and c["e_frob"] <= gate, (A.shape, k, c)


def test_batched_uneven_fp32_and_mixed():
    ws = _uneven(8, 1500, 48, seed=5)
    As = [torch.tensor(w.A.astype(np.float32), device=DEV) for w in ws]
    ref = [oracle.hsvd(w.A.astype(np.float32).astype(np.float64), w.p, w.q, w.k, 0.0) for w in ws]
    for mixed, gate in ((False, 1e-5), (True, 1e-3)):
        print("batched f32 mixed" if mixed else "batched f32", flush=True)
        outs = H.svd_batched(As, [w.p for w in ws], [w.q for w in ws], [w.k for w in ws], mixed=mixed)
        torch.cuda.synchronize()
        for w, (U, S, Vt, r), (Uo, so, Vto, ro) in zip(ws, outs, ref):
            assert r == ro
            c = metrics.compare(U.double().cpu().numpy(), S.double().cpu().numpy(),
                                Vt.double().cpu().numpy(), r, Uo, so, Vto, ro)
            assert c["e_frob"] <= gate and c["e_sigma"] <= gate, (w.name, mixed, c)


def test_batch_of_one_equals_single_plan():
    """A batched plan over one matrix is the single-matrix plan, bit for bit."""
    w = synth.config0(0)
    A = torch.tensor(w.A, device=DEV)
    U1, S1, Vt1, r1 = H.svd(A, w.p, w.q, w.k)
    ((U2, S2, Vt2, r2),) = H.svd_batched([A], [w.p], [w.q], [w.k])
    torch.cuda.synchronize()
    assert r1 == r2
    for a, b in ((U1, U2), (S1, S2), (Vt1, Vt2)):
        assert torch.equal(a, b)


def test_batched_plan_reuse_with_new_pointers():
    """Re-executing a batched plan on other buffers (pointer table re-upload)."""
    ws = _uneven(3, 700, 20, seed=8)
    shapes = [(w.A.shape[0], w.A.shape[1], w.p, w.q, w.k) for w in ws]
    plan = H.BatchPlan(shapes)
    res = []
    for scale in (1.0, 2.0):
        As = [torch.tensor(scale * w.A, device=DEV) for w in ws]
        Us = [torch.empty((m, k), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
        Ss = [torch.empty((k,), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
        Vts = [torch.empty((k, n), dtype=torch.float64, device=DEV) for (m, n, _, _, k) in shapes]
        plan.execute(As, Us, Ss, Vts)
        torch.cuda.synchronize()
        res.append([s.cpu().numpy() for s in Ss])
        assert plan.ranks() == [w.k for w in ws]
    for s1, s2 in zip(res[0], res[1]):
        assert np.allclose(2.0 * s1, s2, rtol=1e-12, atol=0)
    plan.close()


@pytest.mark.parametrize("prec,m,p,k", [(H.FP64, 512, 2, 20), (H.MIXED_BF16, 2048, 2, 32), (H.FP32, 1500, 3, 24)])
def test_graph_replays_match_direct_launches(prec, m, p, k):
    """A plan that captured its launches into a hipGraph on the first execute replays
    it on every later execute: across alternating inputs (the pointer table changes),
    with eager device work and synchronisations between the replays, every replay is
    bit-identical to a plan of the same options that launches its kernels one by one."""
    rng = np.random.default_rng(m + k)
    dt = torch.float64 if prec == H.FP64 else torch.float32
    As = []
    for _ in range(2):
        A, *_ = synth.low_rank(rng, m, m, 10.0 ** (-np.arange(k) / (k / 4.0)), noise=1e-9)
        As.append(torch.tensor(A, dtype=dt, device=DEV))
    pg = H.Plan(m, m, p, p, k, 0.0, precision=prec, graph=True)
    pe = H.Plan(m, m, p, p, k, 0.0, precision=prec, graph=False)
    outs = lambda: (torch.empty((m, k), dtype=dt, device=DEV), torch.empty((k,), dtype=dt, device=DEV),
                    torch.empty((k, m), dtype=dt, device=DEV))
    Ug, Sg, Vg = outs()
    Ue, Se, Ve = outs()
    for it in range(4):
        A = As[it % 2]
        print(f"graph replay {it} prec={prec}", flush=True)
        pg.execute(A, Ug, Sg, Vg)
        junk = A.double() @ A.double().T          # eager work between replays
        torch.cuda.synchronize()
        pe.execute(A, Ue, Se, Ve)
        torch.cuda.synchronize()
        assert float(junk[0, 0]) == float(junk[0, 0])
        assert torch.equal(Ug, Ue) and torch.equal(Sg, Se) and torch.equal(Vg, Ve), it
        assert pg.rank() == pe.rank() == k
    pg.close()
    pe.close()


def test_batched_rank_classes_graph_replays_match_direct_launches():
    """A batch whose matrices fall into several rank classes (concurrent branches of the
    captured graph, wide merge cores among them): every replay, across alternating inputs
    with eager work and synchronisations between them, is bit-identical to a plan of the
    same batch that launches its kernels one by one."""
    ws = _uneven(6, 1100, 80, seed=22)
    shapes = [(w.A.shape[0], w.A.shape[1], w.p, w.q, w.k) for w in ws]
    inputs = [[torch.tensor(s * w.A, dtype=torch.float32, device=DEV) for w in ws] for s in (1.0, 0.5)]
    mk = lambda: ([torch.empty((m, k), dtype=torch.float32, device=DEV) for (m, n, _, _, k) in shapes],
                  [torch.empty((k,), dtype=torch.float32, device=DEV) for (m, n, _, _, k) in shapes],
                  [torch.empty((k, n), dtype=torch.float32, device=DEV) for (m, n, _, _, k) in shapes])
    pg = H.BatchPlan(shapes, precision=H.FP32, graph=True)
    pe = H.BatchPlan(shapes, precision=H.FP32, graph=False)
    og, oe = mk(), mk()
    for it in range(4):
        As = inputs[it % 2]
        print(f"batched graph replay {it}", flush=True)
        pg.execute(As, *og)
        junk = As[0].double() @ As[0].double().T
        torch.cuda.synchronize()
        pe.execute(As, *oe)
        torch.cuda.synchronize()
        assert float(junk[0, 0]) == float(junk[0, 0])
        for xg, xe in zip(og, oe):
            for a, b in zip(xg, xe):
                assert torch.equal(a, b), it
        assert pg.ranks() == pe.ranks() == [w.k for w in ws]
    pg.close()
    pe.close()


def test_set_workspace_from_torch_memory():
    """hsvd_set_workspace moves a plan's arena into a torch-allocated buffer: executes
    before and after the move (and after a second move) give bit-identical results; a
    buffer below hsvd_workspace_bytes is refused and leaves the plan working."""
    w = synth.config0(3)
    A = torch.tensor(w.A, dtype=torch.float64, device=DEV)
    m, n = A.shape
    plan = H.Plan(m, n, w.p, w.q, w.k, w.tol)
    outs = lambda: (torch.empty((m, w.k), dtype=torch.float64, device=DEV),
                    torch.empty((w.k,), dtype=torch.float64, device=DEV),
                    torch.empty((w.k, n), dtype=torch.float64, device=DEV))
    U0, S0, V0 = outs()
    plan.execute(A, U0, S0, V0)
    need = plan.workspace_bytes()
    with pytest.raises(H.HsvdError, match="needs"):
        plan.set_workspace(torch.empty(need - 256, dtype=torch.uint8, device=DEV))
    for rep in range(2):
        buf = torch.empty(need + 1024, dtype=torch.uint8, device=DEV)
        plan.set_workspace(buf)
        U1, S1, V1 = outs()
        plan.execute(A, U1, S1, V1)
        torch.cuda.synchronize()
        assert torch.equal(U0, U1) and torch.equal(S0, S1) and torch.equal(V0, V1), rep
    plan.close()


@pytest.mark.parametrize("m,n,p,q,k,order", [(512, 512, 2, 2, 20, H.ORDER_COLS_LAST),
                                             (700, 1300, 5, 3, 12, H.ORDER_ROWS_LAST),
                                             (1300, 700, 3, 5, 12, H.ORDER_COLS_LAST),
                                             (600, 2000, 1, 4, 16, H.ORDER_AUTO),
                                             (2000, 600, 4, 1, 16, H.ORDER_AUTO)])
def test_merge_order_parity_fp64(m, n, p, q, k, order):
    """Both orders of the two sets of merges (Algorithm 1 as printed, and column slabs
    merged last) and the automatic choice, against the oracle's same order; one-direction
    grids (p x 1, 1 x q) included."""
    rng = np.random.default_rng(m + 3 * n + p + q)
    sigma = 10.0 ** (-np.arange(k) / (k / 3.0))
    A, *_ = synth.low_rank(rng, m, n, sigma, noise=1e-9)
    print(f"order {order}: {m}x{n} {p}x{q} k={k}", flush=True)
    check_parity(A, p, q, k, order=order)


def test_merge_order_mixed_and_float32():
    """The opposite order on the float32-storage and mixed paths (short-fat input, auto)."""
    rng = np.random.default_rng(99)
    A, *_ = synth.low_rank(rng, 1024, 3072, 10.0 ** (-np.arange(24) / 8.0), noise=1e-6)
    check_parity(A, 2, 6, 24, dtype=torch.float32, gate=1e-5)
    Uo, so, Vto, ro = oracle.hsvd(A.astype(np.float32).astype(np.float64), 2, 6, 24, 0.0, order="cols_last")
    Ug, sg, Vtg, rg = run_gpu(A, 2, 6, 24, 0.0, torch.float32, mixed=True)
    c = metrics.compare(Ug, sg, Vtg, rg, Uo, so, Vto, ro)
    print("mixed cols_last", c, flush=True)
    assert rg == ro and c["e_frob"] <= 1e-3


# ----------------------------------------------------------------------------- Gram input
def check_gram(X, p, q, k, tol=0.0, dtype=torch.float64, gate=1e-9, refine=0, refine_eps=None, **opts):
    Xo = X if dtype == torch.float64 else X.astype(np.float32).astype(np.float64)
    info = {}
    Uo, so, Vto, ro = oracle.hsvd_gram(Xo, p, q, k, tol, refine=refine, refine_eps=refine_eps, info=info)
    Xt = torch.tensor(X, dtype=dtype, device=DEV)
    plan = H.Plan(X.shape[0], X.shape[1], p, q, k, tol, gram=True, refine_steps=refine,
                  refine_eps=refine_eps or 0.0,
                  precision=H.FP64 if dtype == torch.float64 else H.FP32, **opts)
    U = torch.empty((X.shape[0], k), dtype=dtype, device=DEV)
    S = torch.empty((k,), dtype=dtype, device=DEV)
    Vt = torch.empty((k, X.shape[1]), dtype=dtype, device=DEV)
    plan.execute(Xt, U, S, Vt)
    rg = plan.rank()
    assert plan.status() & 0xFFFF == 0
    if refine_eps:
        assert plan.refine_iterations() == info["refine_iterations"]
    plan.close()
    Ug, sg, Vtg = (t.double().cpu().numpy() for t in (U, S, Vt))
    assert rg == ro, (rg, ro)
    c = metrics.compare(Ug, sg, Vtg, rg, Uo, so, Vto, ro)
    print(f"gram {X.shape} {p}x{q} k={k}", c, flush=True)
    assert c["e_sigma"] <= gate and c["e_frob"] <= gate
    assert np.all(sg[rg:] == 0) and np.all(Ug[:, rg:] == 0) and np.all(Vtg[rg:] == 0)
    for i in range(rg):
        j = np.argmax(np.abs(Ug[:, i]))
        assert Ug[j, i] > 0
    return c


@pytest.mark.parametrize("m,n,p,q,k", [(3000, 300, 3, 2, 12), (20000, 256, 4, 4, 25),
                                       (700, 200, 2, 3, 10), (150, 400, 4, 4, 16)])
def test_gram_parity_fp64(m, n, p, q, k):
    """Gram plans (X^T X formed on the device, trees on it, projection of X) against the
    oracle's Gram reading: tall X with several row chunks of partial Grams, an n that is
    not a multiple of the 64-wide Gram tiles, and a short-fat X whose Gram is rank-deficient."""
    rng = np.random.default_rng(m + n + k)
    sigma = 10.0 ** (-np.arange(k) / (k / 3.0))
    X, *_ = synth.low_rank(rng, m, n, sigma, noise=1e-9)
    c = check_gram(X, p, q, k)
    assert c["sin_u"] <= 1e-8 and c["sin_v"] <= 1e-8


def test_gram_tol_refinement_and_float32():
    """tol on X^T X's values, Algorithm 2 on X (fixed count and to a tolerance), and the
    float32-storage path of a Gram plan."""
    rng = np.random.default_rng(41)
    X, *_ = synth.low_rank(rng, 2500, 320, 10.0 ** (-np.arange(20) / 4.0), noise=1e-6)
    check_gram(X, 2, 4, 20, tol=1e-6)
    check_gram(X, 4, 4, 12, refine=2)
    check_gram(X, 4, 4, 12, refine=6, refine_eps=1e-6)
    check_gram(X, 2, 2, 12, dtype=torch.float32, gate=1e-5)


def test_gram_plan_reuse_and_errors():
    """A Gram plan re-forms X^T X on every execute (a second input of the same shape
    gives that input's factors); mixed precision is refused."""
    rng = np.random.default_rng(43)
    plan = H.Plan(1200, 256, 2, 2, 10, gram=True)
    outs = []
    for s in (0, 1):
        X, *_ = synth.low_rank(rng, 1200, 256, (1.0 + s) * 10.0 ** (-np.arange(10) / (3.0 + s)), noise=1e-8)
        U = torch.empty((1200, 10), dtype=torch.float64, device=DEV)
        S = torch.empty((10,), dtype=torch.float64, device=DEV)
        Vt = torch.empty((10, 256), dtype=torch.float64, device=DEV)
        plan.execute(torch.tensor(X, device=DEV), U, S, Vt)
        torch.cuda.synchronize()
        so = oracle.hsvd_gram(X, 2, 2, 10)[1]
        assert np.max(np.abs(S.cpu().numpy() - so)) <= 1e-9 * so[0]
        outs.append(S.cpu().numpy())
    assert np.max(np.abs(outs[0] - outs[1])) > 1e-3
    plan.close()
    with pytest.raises(H.HsvdError):
        H.Plan(1200, 256, 2, 2, 10, gram=True, precision=H.MIXED_BF16)
    with pytest.raises(H.HsvdError):
        H.Plan(1200, 256, 300, 2, 10, gram=True)


# ----------------------------------------------------------------------------- launch-shape tunables
@pytest.mark.parametrize("thin_rows,merge_qr,leaf_qr", [(64, 0, 0), (512, 0, 1), (128, 1, 2), (128, 2, 1),
                                                         (256, 3, 2)])
def test_tunables_keep_parity(thin_rows, merge_qr, leaf_qr):
    """Chunk rows of the thin products, the panel-QR merge path (column merges, row
    merges, both) and the leaves' QR (panel QR, chunked TSQR) change the launch shapes
    only: every setting meets the float64 gate."""
    rng = np.random.default_rng(60 + thin_rows + merge_qr)
    A, *_ = synth.low_rank(rng, 1500, 1100, 10.0 ** (-np.arange(16) / 5.0), noise=1e-9)
    check_parity(A, 3, 4, 16, thin_rows=thin_rows, merge_qr=merge_qr, leaf_qr=leaf_qr)


def test_autotune_matches_an_explicit_plan(tmp_path, monkeypatch):
    """An autotuned plan reports its choice, records it in HSVD_TUNE_CACHE, and gives the
    same bits as a plan made with the chosen values; the result meets the gate."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HSVD_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(61)
    A, *_ = synth.low_rank(rng, 2304, 1536, 10.0 ** (-np.arange(20) / 6.0), noise=1e-9)
    At = torch.tensor(A, device=DEV)
    m, n = A.shape
    outs = []
    tp = H.Plan(m, n, 4, 3, 20, autotune=True)
    tu = tp.tuning()
    print("tuning", tu, flush=True)
    assert tu["tuned"] and tu["thin_rows"] in (128, 256, 512) and 0 <= tu["merge_qr"] <= 3
    lines = cache.read_text().split("\n")
    assert any(ln.split()[1:4] == [str(tu["thin_rows"] if tu["thin_rows"] != 128 else 0), str(tu["merge_qr"]),
                                   str(tu["leaf_qr"])]
               for ln in lines if ln.strip())
    ep = H.Plan(m, n, 4, 3, 20, thin_rows=tu["thin_rows"], merge_qr=tu["merge_qr"], leaf_qr=tu["leaf_qr"])
    for plan in (tp, ep):
        U = torch.empty((m, 20), dtype=torch.float64, device=DEV)
        S = torch.empty((20,), dtype=torch.float64, device=DEV)
        Vt = torch.empty((20, n), dtype=torch.float64, device=DEV)
        plan.execute(At, U, S, Vt)
        torch.cuda.synchronize()
        outs.append((U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), plan.rank()))
        plan.close()
    assert outs[0][3] == outs[1][3]
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    Uo, so, Vto, ro = oracle.hsvd(A, 4, 3, 20)
    c = metrics.compare(*outs[0], Uo, so, Vto, ro)
    assert c["e_sigma"] <= 1e-10 and c["e_frob"] <= 1e-10
