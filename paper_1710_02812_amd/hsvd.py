"""ctypes binding of libhsvd.so (include/hsvd.h, include/hsvd_debug.h).

Argument marshalling only: every step of the method runs in the HIP library.
Tensors are PyTorch-ROCm device tensors; the current torch stream is passed as
the hipStream_t.  The library is loaded on first use and a missing or stale
build raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsvd.so")

HSVD_OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_INVALID", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_NONFINITE",
                5: "ERR_NOCONV", 6: "ERR_UNSUPPORTED"}
FP64, FP32, MIXED_BF16 = 0, 1, 2
RULE_GAMMA, RULE_FROB = 0, 1
ORDER_AUTO, ORDER_ROWS_LAST, ORDER_COLS_LAST = 0, 1, 2
FLAG_RANK_FALLBACK = 4
FLAG_NONFINITE, FLAG_NOCONV = 0x1, 0x2

EXPORTED = ["hsvd_default_options", "hsvd_plan", "hsvd_plan_ex", "hsvd_execute", "hsvd_destroy",
            "hsvd_get_rank", "hsvd_get_status", "hsvd_workspace_bytes", "hsvd_last_error",
            "hsvd_get_refine_iterations",
            "hsvd_set_profiling", "hsvd_launch_times", "hsvd_launch_work",
            "hsvd_plan_batched", "hsvd_execute_batched", "hsvd_get_ranks",
            "hsvd_features_plan", "hsvd_features_execute", "hsvd_plan_widths", "hsvd_get_leaf_info",
            "hsvd_rank_model_create", "hsvd_rank_model_destroy", "hsvd_rank_model_set_params",
            "hsvd_rank_model_get_params", "hsvd_rank_model_train", "hsvd_rank_model_grad",
            "hsvd_rank_model_predict",
            "hsvd_debug_jacobi", "hsvd_debug_tsqr", "hsvd_debug_cholqr", "hsvd_debug_panel_qr",
            "hsvd_debug_plan_check", "hsvd_svd_static", "hsvd_set_workspace", "hsvd_set_rank_model",
            "hsvd_get_leaf_widths", "hsvd_plan_gram", "hsvd_get_tuning",
            "hsvd_debug_gemm", "hsvd_debug_probe",
            "hsvd_debug_plan_check_batched"]
LAUNCH_KINDS = ["gemm_ax", "gemm_atx", "tsqr_factor", "tsqr_apply", "gram", "reduce", "thin_nn",
                "sum", "core", "output", "gemm_ax_bf16", "gemm_atx_bf16", "energy", "features", "cholqr",
                "check", "panel_qr", "gemm_ax_f32", "gemm_atx_f32", "gram_xtx", "core_wide"]


class HsvdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("power_steps", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("refine_eps", ctypes.c_double),
                ("graph", ctypes.c_int32), ("order", ctypes.c_int32),
                ("thin_rows", ctypes.c_int32), ("merge_qr", ctypes.c_int32),
                ("leaf_qr", ctypes.c_int32), ("autotune", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libhsvd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1710_02812_amd.build.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.hsvd_default_options.argtypes = [P(Options)]
    L.hsvd_plan.argtypes = [P(vp), i64, i64, i32, i32, i32, f64]
    L.hsvd_plan_ex.argtypes = [P(vp), i64, i64, i32, i32, i32, f64, P(Options)]
    L.hsvd_execute.argtypes = [vp, vp, vp, vp, vp, vp]
    L.hsvd_destroy.argtypes = [vp]
    L.hsvd_get_rank.argtypes = [vp, P(i32)]
    L.hsvd_get_refine_iterations.argtypes = [vp, P(i32)]
    L.hsvd_get_status.argtypes = [vp, P(ctypes.c_uint32)]
    L.hsvd_workspace_bytes.argtypes = [vp, P(ctypes.c_size_t)]
    L.hsvd_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    L.hsvd_set_rank_model.argtypes = [vp, vp, ctypes.c_size_t]
    L.hsvd_plan_gram.argtypes = [P(vp), i64, i64, i32, i32, i32, f64, P(Options)]
    L.hsvd_get_tuning.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(ctypes.c_float)]
    L.hsvd_get_leaf_widths.argtypes = [vp, P(i32), i32, P(i32), P(i32)]
    L.hsvd_last_error.restype = ctypes.c_char_p
    L.hsvd_set_profiling.argtypes = [vp, i32]
    L.hsvd_launch_times.argtypes = [vp, P(i32), P(ctypes.c_float), i32, P(i32)]
    L.hsvd_launch_work.argtypes = [vp, P(f64), P(f64), i32, P(i32)]
    L.hsvd_plan_batched.argtypes = [P(vp), i32, P(i64), P(i64), P(i32), P(i32), P(i32), f64, P(Options)]
    L.hsvd_execute_batched.argtypes = [vp, P(vp), P(vp), P(vp), P(vp), vp]
    L.hsvd_get_ranks.argtypes = [vp, P(i32), i32]
    u64 = ctypes.c_uint64
    L.hsvd_features_plan.argtypes = [P(vp), i64, i64, i32, i32, i32, u64]
    L.hsvd_features_execute.argtypes = [vp, vp, vp, vp]
    L.hsvd_plan_widths.argtypes = [P(vp), i64, i64, i32, i32, i32, f64, P(Options), P(i32)]
    L.hsvd_get_leaf_info.argtypes = [vp, P(i32), P(i32), i32]
    L.hsvd_rank_model_create.argtypes = [P(vp), u64]
    L.hsvd_rank_model_destroy.argtypes = [vp]
    L.hsvd_rank_model_set_params.argtypes = [vp, P(ctypes.c_float), i32]
    L.hsvd_rank_model_get_params.argtypes = [vp, P(ctypes.c_float), i32]
    L.hsvd_rank_model_train.argtypes = [vp, vp, vp, i32, i32, ctypes.c_float, vp, vp]
    L.hsvd_rank_model_grad.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    L.hsvd_rank_model_predict.argtypes = [vp, vp, i32, vp, vp]
    L.hsvd_debug_plan_check_batched.argtypes = [i32, P(i64), P(i64), P(i32), P(i32), P(i32), f64,
                                                P(Options), P(ctypes.c_size_t)]
    L.hsvd_debug_jacobi.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, P(ctypes.c_uint32), vp]
    L.hsvd_debug_tsqr.argtypes = [vp, i32, i64, i32, vp, vp, vp]
    L.hsvd_debug_cholqr.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp]
    L.hsvd_debug_panel_qr.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp]
    L.hsvd_debug_gemm.argtypes = [i32, i32, i32, vp, i64, i64, i64, vp, i32, vp, vp]
    L.hsvd_debug_probe.argtypes = [i32, vp, i64, i32, P(f64), P(f64), vp]
    L.hsvd_debug_plan_check.argtypes = [i64, i64, i32, i32, i32, f64, P(Options),
                                        P(ctypes.c_size_t)]
    L.hsvd_svd_static.argtypes = [i64, i64, i32, i32, i32, f64, P(Options), vp, vp, vp, vp, P(i32), vp]
    for name in EXPORTED:
        if name != "hsvd_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != HSVD_OK:
        raise HsvdError(status, lib().hsvd_last_error().decode())


def default_options() -> Options:
    o = Options()
    _check(lib().hsvd_default_options(ctypes.byref(o)))
    return o


def _stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _options(precision, rule, oversample, power_steps, refine_steps, max_sweeps, seed,
             refine_eps: float = 0.0) -> Options:
    o = default_options()
    o.precision = precision
    o.rule = rule
    if oversample is not None:
        o.oversample = oversample
    if power_steps is not None:
        o.power_steps = power_steps
    o.refine_steps = refine_steps
    if max_sweeps is not None:
        o.max_sweeps = max_sweeps
    o.seed = seed
    o.refine_eps = float(refine_eps)
    return o


class Plan:
    """Owns an hsvd_plan_t.  Create once per shape; execute many times."""

    def __init__(self, m: int, n: int, p: int, q: int, k: int, tol: float = 0.0, *,
                 precision: int = FP64, rule: int = RULE_GAMMA, oversample: int | None = None,
                 power_steps: int | None = None, refine_steps: int = 0,
                 max_sweeps: int | None = None, seed: int = 0, leaf_widths=None,
                 refine_eps: float = 0.0, graph: bool = True, order: int = ORDER_AUTO, gram: bool = False,
                 thin_rows: int = 0, merge_qr: int = 0, leaf_qr: int = 0, autotune: bool = False):
        """leaf_widths: optional p x q per-block sketch widths (hsvd_plan_widths);
        graph: replay a hipGraph captured on the first execute; order: ORDER_AUTO,
        ORDER_ROWS_LAST (Algorithm 1 as printed) or ORDER_COLS_LAST (the opposite order);
        gram: decompose X^T X (p x q grid of the n x n Gram matrix; hsvd_plan_gram);
        thin_rows, merge_qr: launch-shape tunables; autotune: let the plan time and pick them."""
        o = default_options()
        o.graph = 1 if graph else 0
        o.order = order
        o.thin_rows = thin_rows
        o.merge_qr = merge_qr
        o.leaf_qr = leaf_qr
        o.autotune = 1 if autotune else 0
        o.precision = precision
        o.rule = rule
        if oversample is not None:
            o.oversample = oversample
        if power_steps is not None:
            o.power_steps = power_steps
        o.refine_steps = refine_steps
        if max_sweeps is not None:
            o.max_sweeps = max_sweeps
        o.seed = seed
        o.refine_eps = float(refine_eps)
        h = ctypes.c_void_p()
        if gram:
            if leaf_widths is not None:
                raise ValueError("Gram plans take no leaf widths")
            _check(lib().hsvd_plan_gram(ctypes.byref(h), m, n, p, q, k, float(tol), ctypes.byref(o)))
        elif leaf_widths is None:
            _check(lib().hsvd_plan_ex(ctypes.byref(h), m, n, p, q, k, float(tol), ctypes.byref(o)))
        else:
            wv = [int(x) for x in list(np.asarray(leaf_widths).reshape(-1))]
            if len(wv) != p * q:
                raise ValueError("leaf_widths needs p * q entries")
            _check(lib().hsvd_plan_widths(ctypes.byref(h), m, n, p, q, k, float(tol), ctypes.byref(o),
                                          (ctypes.c_int32 * (p * q))(*wv)))
        self._h = h
        self.m, self.n, self.p, self.q, self.k, self.tol = m, n, p, q, k, tol
        self.precision = precision

    def execute(self, A, U, S, Vt, stream=None):
        """Enqueues the method on A (torch device tensors; no synchronisation)."""
        import torch
        dt = torch.float64 if self.precision == FP64 else torch.float32
        for name, t, shape in (("A", A, (self.m, self.n)), ("U", U, (self.m, self.k)),
                               ("S", S, (self.k,)), ("Vt", Vt, (self.k, self.n))):
            if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name}: need a contiguous {dt} device tensor of shape {shape}")
        _check(lib().hsvd_execute(self._h, A.data_ptr(), U.data_ptr(), S.data_ptr(),
                                  Vt.data_ptr(), _stream_handle(stream)))

    def rank(self) -> int:
        r = ctypes.c_int32()
        _check(lib().hsvd_get_rank(self._h, ctypes.byref(r)))
        return r.value

    def tuning(self) -> dict:
        """thin_rows, merge_qr, leaf_qr the plan runs with; tuned, tuned_ms (hsvd_get_tuning)."""
        tr, mq, lq, tu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_float()
        _check(lib().hsvd_get_tuning(self._h, ctypes.byref(tr), ctypes.byref(mq), ctypes.byref(lq),
                                     ctypes.byref(tu), ctypes.byref(ms)))
        return {"thin_rows": tr.value, "merge_qr": mq.value, "leaf_qr": lq.value, "tuned": bool(tu.value),
                "tuned_ms": ms.value}

    def refine_iterations(self) -> int:
        """Algorithm 2 iterations the last execute ran (hsvd_get_refine_iterations)."""
        r = ctypes.c_int32()
        _check(lib().hsvd_get_refine_iterations(self._h, ctypes.byref(r)))
        return r.value

    def leaf_info(self):
        """(ranks, fallback flags) of the leaves, p x q int arrays."""
        c = self.p * self.q
        r = (ctypes.c_int32 * c)()
        f = (ctypes.c_int32 * c)()
        _check(lib().hsvd_get_leaf_info(self._h, r, f, c))
        return (np.array(list(r), dtype=np.int32).reshape(self.p, self.q),
                np.array(list(f), dtype=np.int32).reshape(self.p, self.q))

    def status(self) -> int:
        f = ctypes.c_uint32()
        _check(lib().hsvd_get_status(self._h, ctypes.byref(f)))
        return f.value

    def set_profiling(self, enable: bool = True):
        _check(lib().hsvd_set_profiling(self._h, 1 if enable else 0))

    def launch_times(self):
        """[(kind name, ms)] for every launch of the last profiled execute."""
        n = ctypes.c_int32()
        _check(lib().hsvd_launch_times(self._h, None, None, 0, ctypes.byref(n)))
        kinds = (ctypes.c_int32 * n.value)()
        ms = (ctypes.c_float * n.value)()
        _check(lib().hsvd_launch_times(self._h, kinds, ms, n.value, ctypes.byref(n)))
        return [(LAUNCH_KINDS[kinds[i]], float(ms[i])) for i in range(n.value)]

    def launch_work(self):
        """[(flops, bytes)]: algorithmic work of every launch of one execute, in the
        order of launch_times (host only)."""
        n = ctypes.c_int32()
        _check(lib().hsvd_launch_work(self._h, None, None, 0, ctypes.byref(n)))
        f = (ctypes.c_double * n.value)()
        b = (ctypes.c_double * n.value)()
        _check(lib().hsvd_launch_work(self._h, f, b, n.value, ctypes.byref(n)))
        return [(float(f[i]), float(b[i])) for i in range(n.value)]

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().hsvd_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def set_rank_model(self, model):
        """Attaches a RankModel's current parameters (None detaches): later executes
        take the learned path (hsvd_set_rank_model)."""
        if model is None:
            _check(lib().hsvd_set_rank_model(self._h, None, 0))
            return
        theta = model.params() if isinstance(model, RankModel) else np.asarray(model, dtype=np.float32)
        buf = (ctypes.c_float * theta.size)(*theta.ravel().tolist())
        _check(lib().hsvd_set_rank_model(self._h, buf, 4 * theta.size))

    def leaf_widths(self):
        """(p x q widths, refits, plain) of the last learned execute (hsvd_get_leaf_widths)."""
        c = self.p * self.q
        w = (ctypes.c_int32 * c)()
        rf, pl = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().hsvd_get_leaf_widths(self._h, w, c, ctypes.byref(rf), ctypes.byref(pl)))
        return np.array(list(w), dtype=np.int32).reshape(self.p, self.q), rf.value, pl.value

    def set_workspace(self, buf):
        """Moves the plan's workspace into `buf`, a device tensor (any dtype) of at least
        workspace_bytes() bytes whose storage is 256-byte aligned; keep it alive until
        close()."""
        self._ws_buf = buf
        _check(lib().hsvd_set_workspace(self._h, buf.data_ptr(), buf.numel() * buf.element_size()))

    def close(self):
        if getattr(self, "_h", None):
            lib().hsvd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_features(A, p: int, q: int, seed: int = 0):
    """Learned-rank features of every block of a torch device matrix (float64 or
    float32): a (p * q, 16) float32 device tensor, row i * q + j for block (i, j)."""
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A must be float64 or float32")
    A = A.contiguous()
    m, n = A.shape
    h = ctypes.c_void_p()
    _check(lib().hsvd_features_plan(ctypes.byref(h), m, n, p, q, FP64 if A.dtype == torch.float64 else FP32,
                                    seed))
    F = torch.empty((p * q, 16), dtype=torch.float32, device=A.device)
    try:
        _check(lib().hsvd_features_execute(h, A.data_ptr(), F.data_ptr(), _stream_handle()))
        torch.cuda.synchronize()
    finally:
        lib().hsvd_destroy(h)
    return F


class RankModel:
    """The learned block-rank network (hsvd_rank_model_*): trained and evaluated on
    the GPU by the library's own kernels."""
    N_PARAMS = 5313

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hsvd_rank_model_create(ctypes.byref(h), seed))
        self._h = h

    def params(self) -> np.ndarray:
        buf = (ctypes.c_float * self.N_PARAMS)()
        _check(lib().hsvd_rank_model_get_params(self._h, buf, self.N_PARAMS))
        return np.array(list(buf), dtype=np.float32)

    def set_params(self, theta):
        theta = np.asarray(theta, dtype=np.float32).ravel()
        buf = (ctypes.c_float * self.N_PARAMS)(*theta.tolist())
        _check(lib().hsvd_rank_model_set_params(self._h, buf, self.N_PARAMS))

    def train(self, X, T, steps: int, lr: float = 3e-3):
        """Adam steps on (features X (count, 16), targets T (count,)) float32 device
        tensors; returns the per-step minibatch losses (device tensor)."""
        import torch
        X = X.contiguous().float()
        T = T.contiguous().float()
        losses = torch.empty((steps,), dtype=torch.float32, device=X.device)
        _check(lib().hsvd_rank_model_train(self._h, X.data_ptr(), T.data_ptr(), X.shape[0], steps, lr,
                                           losses.data_ptr(), _stream_handle()))
        return losses

    def grad(self, X, T, batch_index: int = 0):
        import torch
        X = X.contiguous().float()
        T = T.contiguous().float()
        g = torch.empty((self.N_PARAMS,), dtype=torch.float32, device=X.device)
        L = torch.empty((1,), dtype=torch.float32, device=X.device)
        _check(lib().hsvd_rank_model_grad(self._h, X.data_ptr(), T.data_ptr(), X.shape[0], batch_index,
                                          g.data_ptr(), L.data_ptr(), _stream_handle()))
        return g, L

    def predict(self, X):
        import torch
        X = X.contiguous().float()
        out = torch.empty((X.shape[0],), dtype=torch.float32, device=X.device)
        _check(lib().hsvd_rank_model_predict(self._h, X.data_ptr(), X.shape[0], out.data_ptr(),
                                             _stream_handle()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().hsvd_rank_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def learned_svd(A, p: int, q: int, k: int, tol: float, model: "RankModel", **opts):
    """Hierarchical SVD with the learned sketch widths (a plan with the model attached:
    features, prediction, widths, refits and the plain-width fallback all run in the
    library).  Returns (U, S, Vt, r, info) with info = widths, refits, plain, leaf ranks
    and fallback flags of the run that produced the output."""
    import torch
    A = A.contiguous()
    m, n = A.shape
    prec = FP64 if A.dtype == torch.float64 else FP32
    opts.setdefault("rule", RULE_FROB)
    plan = Plan(m, n, p, q, k, tol, precision=prec, **opts)
    plan.set_rank_model(model)
    U = torch.empty((m, k), dtype=A.dtype, device=A.device)
    S = torch.empty((k,), dtype=A.dtype, device=A.device)
    Vt = torch.empty((k, n), dtype=A.dtype, device=A.device)
    plan.execute(A, U, S, Vt)
    r = plan.rank()
    widths, refits, plain = plan.leaf_widths()
    ranks, fb = plan.leaf_info()
    flags = plan.status() & 0xFFFF
    plan.close()
    if flags & ~FLAG_RANK_FALLBACK:
        raise HsvdError(5 if flags & FLAG_NOCONV else 4, f"device status flags {flags:#x}")
    info = {"widths": widths, "refits": refits, "plain": plain, "leaf_ranks": ranks, "fallback": fb}
    return U, S, Vt, r, info


class BatchPlan:
    """Owns an hsvd_plan_t over several matrices of different shapes
    (hsvd_plan_batched): one execute runs every stage of all of them together."""

    def __init__(self, shapes, tol: float = 0.0, *, precision: int = FP64, rule: int = RULE_GAMMA,
                 oversample: int | None = None, power_steps: int | None = None,
                 refine_steps: int = 0, max_sweeps: int | None = None, seed: int = 0,
                 refine_eps: float = 0.0, thin_rows: int = 0, merge_qr: int = 0, leaf_qr: int = 0,
                 autotune: bool = False, graph: bool = True):
        """shapes: list of (m, n, p, q, k); thin_rows, merge_qr, leaf_qr: launch-shape
        tunables (0: defaults); autotune: let the plan time and pick them; graph: replay a
        hipGraph captured on the first execute."""
        c = len(shapes)
        i64a, i32a = ctypes.c_int64 * c, ctypes.c_int32 * c
        ms = i64a(*[s[0] for s in shapes])
        ns = i64a(*[s[1] for s in shapes])
        ps = i32a(*[s[2] for s in shapes])
        qs = i32a(*[s[3] for s in shapes])
        ks = i32a(*[s[4] for s in shapes])
        o = _options(precision, rule, oversample, power_steps, refine_steps, max_sweeps, seed,
                     refine_eps)
        o.thin_rows, o.merge_qr, o.leaf_qr = thin_rows, merge_qr, leaf_qr
        o.autotune = 1 if autotune else 0
        o.graph = 1 if graph else 0
        h = ctypes.c_void_p()
        _check(lib().hsvd_plan_batched(ctypes.byref(h), c, ms, ns, ps, qs, ks, float(tol), ctypes.byref(o)))
        self._h = h
        self.shapes = [tuple(s) for s in shapes]
        self.precision = precision

    def tuning(self) -> dict:
        """thin_rows, merge_qr, leaf_qr the plan runs with; tuned, tuned_ms (hsvd_get_tuning)."""
        return Plan.tuning(self)

    def execute(self, As, Us, Ss, Vts, stream=None):
        """Enqueues the method on every matrix (lists of torch device tensors)."""
        import torch
        dt = torch.float64 if self.precision == FP64 else torch.float32
        c = len(self.shapes)
        if not (len(As) == len(Us) == len(Ss) == len(Vts) == c):
            raise ValueError("one A, U, S, Vt per matrix")
        for i, (m, n, _, _, k) in enumerate(self.shapes):
            for name, t, shape in (("A", As[i], (m, n)), ("U", Us[i], (m, k)), ("S", Ss[i], (k,)),
                                   ("Vt", Vts[i], (k, n))):
                if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous() or not t.is_cuda:
                    raise ValueError(f"{name}[{i}]: need a contiguous {dt} device tensor of shape {shape}")
        arr = ctypes.c_void_p * c
        _check(lib().hsvd_execute_batched(self._h, arr(*[t.data_ptr() for t in As]),
                                          arr(*[t.data_ptr() for t in Us]), arr(*[t.data_ptr() for t in Ss]),
                                          arr(*[t.data_ptr() for t in Vts]), _stream_handle(stream)))

    def ranks(self):
        c = len(self.shapes)
        r = (ctypes.c_int32 * c)()
        _check(lib().hsvd_get_ranks(self._h, r, c))
        return list(r)

    def refine_iterations(self) -> int:
        """Algorithm 2 iterations the last execute ran (one count for the whole batch)."""
        r = ctypes.c_int32()
        _check(lib().hsvd_get_refine_iterations(self._h, ctypes.byref(r)))
        return r.value

    def status(self) -> int:
        f = ctypes.c_uint32()
        _check(lib().hsvd_get_status(self._h, ctypes.byref(f)))
        return f.value

    def set_profiling(self, enable: bool = True):
        _check(lib().hsvd_set_profiling(self._h, 1 if enable else 0))

    def launch_times(self):
        return Plan.launch_times(self)

    def launch_work(self):
        return Plan.launch_work(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().hsvd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def svd_batched(As, ps, qs, ks, tol: float = 0.0, mixed: bool = False, **opts):
    """Hierarchical MAT truncated SVDs of a list of torch device matrices in one
    batched plan.  Returns a list of (U, S, Vt, r)."""
    import torch
    dt = As[0].dtype
    if any(A.dtype != dt for A in As) or dt not in (torch.float64, torch.float32):
        raise ValueError("all matrices must share a float64 or float32 dtype")
    prec = FP64 if dt == torch.float64 else (MIXED_BF16 if mixed else FP32)
    As = [A.contiguous() for A in As]
    shapes = [(A.shape[0], A.shape[1], p, q, k) for A, p, q, k in zip(As, ps, qs, ks)]
    plan = BatchPlan(shapes, tol, precision=prec, **opts)
    Us = [torch.empty((m, k), dtype=dt, device=As[0].device) for (m, n, _, _, k) in shapes]
    Ss = [torch.empty((k,), dtype=dt, device=As[0].device) for (m, n, _, _, k) in shapes]
    Vts = [torch.empty((k, n), dtype=dt, device=As[0].device) for (m, n, _, _, k) in shapes]
    plan.execute(As, Us, Ss, Vts)
    rs = plan.ranks()
    flags = plan.status()
    plan.close()
    flags &= 0xFFFF
    if flags:
        raise HsvdError(5 if flags & FLAG_NOCONV else 4, f"device status flags {flags:#x}")
    return [(U, S, Vt, r) for U, S, Vt, r in zip(Us, Ss, Vts, rs)]


def svd(A, p: int, q: int, k: int, tol: float = 0.0, mixed: bool = False, **opts):
    """Hierarchical MAT truncated SVD of a torch device matrix A (float64 or float32;
    mixed=True selects the bfloat16 matrix-core passes for a float32 A).

    Returns (U [m x k], S [k], Vt [k x n], r); entries past the rank r are zero.
    """
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A must be float64 or float32")
    if mixed and A.dtype != torch.float32:
        raise ValueError("the mixed path takes a float32 A")
    prec = FP64 if A.dtype == torch.float64 else (MIXED_BF16 if mixed else FP32)
    A = A.contiguous()
    m, n = A.shape
    plan = Plan(m, n, p, q, k, tol, precision=prec, **opts)
    U = torch.empty((m, k), dtype=A.dtype, device=A.device)
    S = torch.empty((k,), dtype=A.dtype, device=A.device)
    Vt = torch.empty((k, n), dtype=A.dtype, device=A.device)
    plan.execute(A, U, S, Vt)
    r = plan.rank()
    flags = plan.status()
    plan.close()
    flags &= 0xFFFF
    if flags:
        raise HsvdError(5 if flags & FLAG_NOCONV else 4, f"device status flags {flags:#x}")
    return U, S, Vt, r


def svd_static(A, p: int, q: int, k: int, tol: float = 0.0, **opts):
    """hsvd_svd_static: the allocation-free one-shot SVD of a torch device matrix
    (float64, or float32 with precision=FP32 / MIXED_BF16).  Returns (U, S, Vt, r); the
    outputs are allocated here by torch, the library itself allocates no device memory.
    Blocking (the call synchronises the current stream)."""
    import torch
    if A.dtype not in (torch.float64, torch.float32) or A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D float64 or float32 device tensor")
    A = A.contiguous()
    m, n = A.shape
    o = _options(opts.pop("precision", FP64 if A.dtype == torch.float64 else FP32),
                 opts.pop("rule", RULE_GAMMA), opts.pop("oversample", None), opts.pop("power_steps", None),
                 opts.pop("refine_steps", 0), opts.pop("max_sweeps", None), opts.pop("seed", 0),
                 opts.pop("refine_eps", 0.0))
    if opts:
        raise TypeError(f"unknown options {sorted(opts)}")
    U = torch.empty((m, k), dtype=A.dtype, device=A.device)
    S = torch.empty((k,), dtype=A.dtype, device=A.device)
    Vt = torch.empty((k, n), dtype=A.dtype, device=A.device)
    r = ctypes.c_int32()
    _check(lib().hsvd_svd_static(m, n, p, q, k, float(tol), ctypes.byref(o), A.data_ptr(), U.data_ptr(),
                                 S.data_ptr(), Vt.data_ptr(), ctypes.byref(r), _stream_handle()))
    return U, S, Vt, r.value


def debug_jacobi(M, max_sweeps: int = 40, with_v: bool = True, precondition: bool = False):
    """Jacobi SVD of a batch of dense square float64 matrices M (batch, n, n);
    precondition=True runs the sweeps on L of M = L Q (left pairs only)."""
    import torch
    b, n, _ = M.shape
    Mc = M.transpose(1, 2).contiguous()       # col-major storage
    U = torch.empty_like(Mc)
    S = torch.empty((b, n), dtype=torch.float64, device=M.device)
    V = torch.empty_like(Mc) if with_v else None
    fl = ctypes.c_uint32()
    _check(lib().hsvd_debug_jacobi(Mc.data_ptr(), b, n, U.data_ptr(), S.data_ptr(),
                                   V.data_ptr() if with_v else None, max_sweeps,
                                   int(precondition), ctypes.byref(fl), _stream_handle()))
    return (U.transpose(1, 2), S, V.transpose(1, 2) if with_v else None, fl.value & 0xFFFF,
            fl.value >> 16)


PROBE_KINDS = {"read": 0, "copy": 1, "mfma_f64": 2, "mfma_bf16": 3, "mfma_f32": 4}


def debug_probe(kind: str, buf=None, iters: int = 0, stream=None):
    """One peak-probe launch (hsvd_debug_probe): (ms, bytes or flops).  buf: a torch
    device tensor for the memory probes (its whole size is streamed)."""
    ms, work = ctypes.c_double(), ctypes.c_double()
    ptr = buf.data_ptr() if buf is not None else None
    nbytes = buf.numel() * buf.element_size() if buf is not None else 0
    _check(lib().hsvd_debug_probe(PROBE_KINDS[kind], ptr, nbytes, iters, ctypes.byref(ms), ctypes.byref(work),
                                  _stream_handle(stream)))
    return ms.value, work.value


def plan_check(m: int, n: int, p: int, q: int, k: int, tol: float = 0.0, **opts) -> int:
    """Builds and bounds-checks a plan on the host only; returns the arena bytes."""
    o = default_options()
    for key, v in opts.items():
        setattr(o, key, v)
    b = ctypes.c_size_t()
    _check(lib().hsvd_debug_plan_check(m, n, p, q, k, float(tol), ctypes.byref(o), ctypes.byref(b)))
    return b.value


def debug_gemm(A, X, op: int = 0, bf16: bool = False, f32: bool = False):
    """One pass product on a single block: op 0 -> A @ X, op 1 -> A.T @ X (float64 result).
    A: (rows, cols) float32/float64 device tensor (row-major); X: float64 (K, N).
    bf16 / f32: the bfloat16 / float32 matrix-core kernels (A float32)."""
    import torch
    rows, cols = A.shape
    K, N = X.shape
    assert K == (cols if op == 0 else rows)
    Ac = A.contiguous()
    Xc = X.t().contiguous()                  # col-major storage
    yr = rows if op == 0 else cols
    Y = torch.empty((N, yr), dtype=torch.float64, device=A.device)
    _check(lib().hsvd_debug_gemm(op, 1 if bf16 else 2 if f32 else 0, int(Ac.dtype == torch.float32), Ac.data_ptr(),
                                 rows, cols, cols, Xc.data_ptr(), N, Y.data_ptr(), _stream_handle()))
    return Y.t()


def plan_check_batched(shapes, tol: float = 0.0, **opts) -> int:
    """Builds and bounds-checks a batched plan on the host only; returns the arena bytes."""
    c = len(shapes)
    i64a, i32a = ctypes.c_int64 * c, ctypes.c_int32 * c
    o = default_options()
    for key, v in opts.items():
        setattr(o, key, v)
    b = ctypes.c_size_t()
    _check(lib().hsvd_debug_plan_check_batched(
        c, i64a(*[s[0] for s in shapes]), i64a(*[s[1] for s in shapes]), i32a(*[s[2] for s in shapes]),
        i32a(*[s[3] for s in shapes]), i32a(*[s[4] for s in shapes]), float(tol), ctypes.byref(o),
        ctypes.byref(b)))
    return b.value


def debug_tsqr(P):
    """TSQR of a batch of float64 panels P (batch, h, w) -> (Q (batch,h,w), R (batch,w,w))."""
    import torch
    b, h, w = P.shape
    Pc = P.transpose(1, 2).contiguous()
    Q = torch.empty_like(Pc)
    R = torch.empty((b, w, w), dtype=torch.float64, device=P.device)
    _check(lib().hsvd_debug_tsqr(Pc.data_ptr(), b, h, w, Q.data_ptr(), R.data_ptr(),
                                 _stream_handle()))
    return Q.transpose(1, 2), R.transpose(1, 2)


def debug_cholqr(P):
    """Cholesky QR (two passes, Householder fallback) of float64 panels P (batch, h, w),
    w <= 64 -> (Q (batch, h, w), R (batch, w, w), fell_back list of 0/1 per panel)."""
    import torch
    b, h, w = P.shape
    Pc = P.transpose(1, 2).contiguous()
    Q = torch.empty_like(Pc)
    R = torch.empty((b, w, w), dtype=torch.float64, device=P.device)
    fb = (ctypes.c_int32 * b)()
    _check(lib().hsvd_debug_cholqr(Pc.data_ptr(), b, h, w, Q.data_ptr(), R.data_ptr(), fb,
                                   _stream_handle()))
    return Q.transpose(1, 2), R.transpose(1, 2), list(fb)


def debug_panel_qr(P):
    """The leaves' one-launch panel QR (repeated Cholesky QR, the first pass shifted;
    Householder where it falls back) of float64 panels P (batch, h, w), w <= 80
    -> (Q (batch, h, w), R (batch, w, w), fell_back list of 0/1 per panel)."""
    import torch
    b, h, w = P.shape
    Pc = P.transpose(1, 2).contiguous()
    Q = torch.empty_like(Pc)
    R = torch.empty((b, w, w), dtype=torch.float64, device=P.device)
    fb = (ctypes.c_int32 * b)()
    _check(lib().hsvd_debug_panel_qr(Pc.data_ptr(), b, h, w, Q.data_ptr(), R.data_ptr(), fb,
                                     _stream_handle()))
    return Q.transpose(1, 2), R.transpose(1, 2), list(fb)
