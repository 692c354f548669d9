"""The allocation-free entry point hsvd_svd_static (device state in a file-scope device
array) against the plan + execute path on the same inputs, on two calls in a row, the
second with a smaller input: outputs bit-identical (same kernels, same schedule, same
seed), ranks equal, and the first also within the float64 gate of the oracle."""
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


def _plan_path(A, p, q, k, tol, **opts):
    m, n = A.shape
    plan = H.Plan(m, n, p, q, k, tol, **opts)
    U = torch.empty((m, k), dtype=A.dtype, device=DEV)
    S = torch.empty((k,), dtype=A.dtype, device=DEV)
    Vt = torch.empty((k, n), dtype=A.dtype, device=DEV)
    plan.execute(A, U, S, Vt)
    r = plan.rank()
    plan.close()
    return U, S, Vt, r


def test_static_entry_matches_plan_path_twice():
    w = synth.config0(0)
    A1 = torch.tensor(w.A, dtype=torch.float64, device=DEV)
    print("static: call 1, 512 x 512 float64, 2 x 2 grid, k = 20", flush=True)
    Us, Ss, Vts, rs = H.svd_static(A1, w.p, w.q, w.k, w.tol)
    Up, Sp, Vtp, rp = _plan_path(A1, w.p, w.q, w.k, w.tol)
    torch.cuda.synchronize()
    assert rs == rp == 20
    assert torch.equal(Us, Up) and torch.equal(Ss, Sp) and torch.equal(Vts, Vtp)
    Uo, so, Vto, ro = oracle.hsvd(w.A, w.p, w.q, w.k, w.tol)
    c = metrics.compare(Us.cpu().numpy(), Ss.cpu().numpy(), Vts.cpu().numpy(), rs, Uo, so, Vto, ro)
    for key in ("e_sigma", "e_frob", "sin_u", "sin_v"):
        assert c[key] <= 1e-10, (key, c)

    rng = np.random.default_rng(11)
    A, *_ = synth.low_rank(rng, 300, 200, 10.0 ** (-np.arange(8) / 3.0), noise=1e-9)
    A2 = torch.tensor(A, dtype=torch.float32, device=DEV)
    print("static: call 2, 300 x 200 float32 storage, 2 x 3 grid, k = 8", flush=True)
    Us, Ss, Vts, rs = H.svd_static(A2, 2, 3, 8, 0.0, precision=H.FP32)
    Up, Sp, Vtp, rp = _plan_path(A2, 2, 3, 8, 0.0, precision=H.FP32)
    torch.cuda.synchronize()
    assert rs == rp == 8
    assert torch.equal(Us, Up) and torch.equal(Ss, Sp) and torch.equal(Vts, Vtp)


def test_static_entry_rejects_large_problems():
    A = torch.zeros((4096, 4096), dtype=torch.float64, device=DEV)
    with pytest.raises(H.HsvdError, match="at most"):
        H.svd_static(A, 4, 4, 64, 0.0)
