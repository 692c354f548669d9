"""Learned block rank on the GPU: the network's kernels against the CPU oracle
(gradients, predictions, Adam), block features by their properties, and what the
trained network gains over the plain method (fewer sketch columns at the same
1e-3 accuracy against the oracle)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import metrics, mlp_oracle as mlp  # noqa: E402
from paper_1710_02812_amd import hsvd as H, synth  # noqa: E402

DEV = "cuda:0"


def _data(count, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((count, mlp.N_IN)).astype(np.float32)
    T = (3.0 + 1.5 * np.tanh(X[:, 0]) + 0.5 * X[:, 3]).astype(np.float32)
    return X, T


@pytest.mark.parametrize("batch_index", [0, 3])
def test_gradient_matches_oracle(batch_index):
    """Backward kernel vs the oracle's gradient at the same float16-rounded weights."""
    X, T = _data(200, 1)
    theta = (mlp.init_params(7) + 0.05 * np.random.default_rng(2).standard_normal(mlp.N_PARAMS)).astype(np.float32)
    model = H.RankModel()
    model.set_params(theta)
    g, L = model.grad(torch.tensor(X, device=DEV), torch.tensor(T, device=DEV), batch_index)
    torch.cuda.synchronize()
    idx = (batch_index * 64 + np.arange(64)) % 200
    L_ref, g_ref = mlp.grad(mlp.fp16(theta), X[idx].astype(np.float64), T[idx].astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    print("grad max err", np.max(np.abs(g - g_ref)), "scale", np.max(np.abs(g_ref)), flush=True)
    assert abs(L.item() - L_ref) <= 1e-5 * max(1.0, L_ref)
    assert np.max(np.abs(g - g_ref)) <= 2e-5 * np.max(np.abs(g_ref))
    model.close()


def test_predict_matches_oracle():
    X, _ = _data(300, 3)
    theta = mlp.init_params(8)
    model = H.RankModel()
    model.set_params(theta)
    y = model.predict(torch.tensor(X, device=DEV)).cpu().numpy()
    y_ref, _ = mlp.forward(mlp.fp16(theta), X.astype(np.float64))
    assert np.max(np.abs(y - y_ref)) <= 1e-5 * max(1.0, np.max(np.abs(y_ref)))
    model.close()


def test_adam_steps_match_oracle():
    """Five training steps on the GPU against the oracle's Adam on the same minibatches."""
    X, T = _data(150, 4)
    theta = mlp.init_params(9)
    model = H.RankModel()
    model.set_params(theta)
    losses = model.train(torch.tensor(X, device=DEV), torch.tensor(T, device=DEV), steps=5, lr=1e-3)
    torch.cuda.synchronize()
    got = model.params().astype(np.float64)
    ref, ref_losses = mlp.train(theta, X.astype(np.float64), T.astype(np.float64), steps=5, lr=1e-3)
    assert np.allclose(losses.cpu().numpy(), ref_losses, rtol=1e-4)
    # Adam moves each weight by about lr * sign(gradient) per step: where a gradient
    # is near zero its float32 and float64 signs may differ, elsewhere they agree
    close = np.abs(got - ref) <= 1e-5
    assert np.mean(close) >= 0.99
    assert np.max(np.abs(got - ref)) <= 2 * 1e-3 * 5
    model.close()


def test_training_reduces_loss_on_gpu():
    X, T = _data(512, 5)
    model = H.RankModel(seed=3)
    Xt, Tt = torch.tensor(X, device=DEV), torch.tensor(T, device=DEV)
    before = model.predict(Xt).cpu().numpy()
    model.train(Xt, Tt, steps=800, lr=3e-3)
    after = model.predict(Xt).cpu().numpy()
    l0 = np.mean((before - T) ** 2) / 2
    l1 = np.mean((after - T) ** 2) / 2
    print("loss", l0, "->", l1, flush=True)
    assert l1 < 0.05 * l0
    model.close()


def test_block_features_properties():
    """Blocks of exact rank r < 16: features past r sit at the floor, the energy
    feature is near 0 (E[||Y||^2] = 16 E), a zero block gives zeros."""
    rng = np.random.default_rng(6)
    m, n, p, q = 512, 768, 2, 3
    A = np.zeros((m, n))
    ranks = [[1, 3, 5], [8, 0, 12]]
    for i in range(p):
        for j in range(q):
            r = ranks[i][j]
            if r == 0:
                continue
            blk = synth.low_rank(rng, 256, 256, np.exp(-np.arange(r) / 2.0))[0]
            A[i * 256:(i + 1) * 256, j * 256:(j + 1) * 256] = blk
    F = H.block_features(torch.tensor(A, device=DEV), p, q).cpu().numpy()
    for i in range(p):
        for j in range(q):
            f = F[i * q + j]
            r = ranks[i][j]
            if r == 0:
                assert np.all(f == 0.0)
                continue
            assert np.all(np.diff(f[:15]) <= 1e-6)                       # descending ratios
            assert np.all(f[r - 1:15] <= -9.0), (r, f)                   # nothing past the rank
            if r > 1:
                assert np.all(f[:r - 1] > -6.0), (r, f)
            assert abs(f[15]) < 1.0


def _field(seed):
    return synth.config4(seed=seed, p=8, q=4, block=512, base_rank=64, max_class=3, k=64)


def _plain_leaf_ranks(w):
    A = torch.tensor(w.A, device=DEV)
    plan = H.Plan(*w.A.shape, w.p, w.q, w.k, w.tol, rule=H.RULE_FROB)
    U = torch.empty((w.A.shape[0], w.k), dtype=torch.float64, device=DEV)
    S = torch.empty((w.k,), dtype=torch.float64, device=DEV)
    Vt = torch.empty((w.k, w.A.shape[1]), dtype=torch.float64, device=DEV)
    plan.execute(A, U, S, Vt)
    ranks, _ = plan.leaf_info()
    out = (U, S, Vt, plan.rank())
    plan.close()
    return ranks, out


def test_learned_rank_gain():
    """Trained on the leaf ranks the method itself chose on four seeded field
    matrices, the network sizes the sketches of a fifth: far fewer columns than
    k + oversample everywhere, same rank, and the 1e-3 error bound against the oracle."""
    Xs, Ts = [], []
    for seed in (10, 11, 12, 13):
        w = _field(seed)
        F = H.block_features(torch.tensor(w.A, device=DEV), w.p, w.q)
        ranks, _ = _plain_leaf_ranks(w)
        Xs.append(F)
        Ts.append(torch.tensor(np.log2(np.maximum(ranks.reshape(-1), 1)).astype(np.float32), device=DEV))
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    model = H.RankModel(seed=1)
    model.train(X, T, steps=1500, lr=3e-3)
    torch.cuda.synchronize()
    w = _field(4)
    A = torch.tensor(w.A, device=DEV)
    U, S, Vt, r, info = H.learned_svd(A, w.p, w.q, w.k, w.tol, model)
    ranks_plain, (U0, S0, Vt0, r0) = _plain_leaf_ranks(w)
    Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, w.tol, "frob")
    c_learned = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), r, Uo, so, Vto, ro)
    c_plain = metrics.compare(U0.cpu().numpy(), S0.cpu().numpy(), Vt0.cpu().numpy(), r0, Uo, so, Vto, ro)
    plain_cols = w.p * w.q * min(w.k + 14, 80)
    learned_cols = int(info["widths"].sum())
    print("learned", c_learned, "plain", c_plain, "columns", learned_cols, "vs", plain_cols,
          "refits", info["refits"], flush=True)
    assert c_plain["e_frob"] <= 1e-3 and c_learned["e_frob"] <= 1e-3
    assert r == ro and r0 == ro
    assert learned_cols <= 0.75 * plain_cols
    # every block got at least the width its true leaf rank needs
    assert np.all(info["widths"] >= ranks_plain)
    assert info["plain"] == 0
    model.close()


def test_learned_path_recovers_from_a_bad_prediction():
    """A network that predicts rank 1 for every block (output weights zero, bias -5:
    sketch width 16) under-sketches the rank-32 blocks: their leaves report the energy
    their sketch missed, the library doubles their widths and runs again, and the
    result still meets the 1e-3 bound against the oracle with the oracle's rank."""
    w = _field(7)
    model = H.RankModel(seed=2)
    theta = model.params()
    theta[5248:5312] = 0.0
    theta[5312] = -5.0
    model.set_params(theta)
    A = torch.tensor(w.A, device=DEV)
    U, S, Vt, r, info = H.learned_svd(A, w.p, w.q, w.k, w.tol, model)
    Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, w.tol, "frob")
    c = metrics.compare(U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), r, Uo, so, Vto, ro)
    print("bad prediction", c, "refits", info["refits"], "plain", info["plain"], flush=True)
    assert info["refits"] >= 1 or info["plain"] == 1
    assert r == ro and c["e_frob"] <= 1e-3
    model.close()


@pytest.mark.parametrize("precision", [H.FP64, H.FP32])
def test_width_plan_energies_from_the_sketch_pass(precision):
    """The leaves' block energies come out of the sketch pass (partial sums per tile).
    Blocks of exact rank below their sketch width (72 and 80 columns: two column tiles
    of the pass, only the first of which counts the block's rows) miss nothing and are
    not flagged; 8-column sketches of blocks of rank 40 and 70 with a flat spectrum miss
    about half their energy and are flagged, the rank-3 block is not, nor the zero block.
    A doubled energy would flag the first case, a halved one would clear the second."""
    rng = np.random.default_rng(11)
    m, n, p, q, bs = 512, 512, 2, 2, 256
    ranks = [[3, 70], [40, 0]]
    A = np.zeros((m, n))
    for i in range(p):
        for j in range(q):
            r = ranks[i][j]
            if r:
                A[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = synth.low_rank(
                    rng, bs, bs, np.exp(-np.arange(r) / 20.0))[0]
    dt = torch.float64 if precision == H.FP64 else torch.float32
    At = torch.tensor(A, device=DEV, dtype=dt)
    k, tol = 80, 1e-3
    out = (torch.empty((m, k), dtype=dt, device=DEV), torch.empty((k,), dtype=dt, device=DEV),
           torch.empty((k, n), dtype=dt, device=DEV))
    for widths, expect in (([[72, 80], [80, 72]], [[0, 0], [0, 0]]),
                           ([[8, 8], [8, 8]], [[0, 1], [1, 0]])):
        plan = H.Plan(m, n, p, q, k, tol, precision=precision, rule=H.RULE_FROB, leaf_widths=widths)
        plan.execute(At, *out)
        torch.cuda.synchronize()
        ranks_got, flags = plan.leaf_info()
        print(precision, widths, ranks_got.tolist(), flags.tolist(), flush=True)
        assert flags.tolist() == expect
        if expect == [[0, 0], [0, 0]]:
            assert ranks_got.tolist() == ranks
        plan.close()
