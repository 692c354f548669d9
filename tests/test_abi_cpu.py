"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the headers declare, and rejects bad arguments before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1710_02812_amd import hsvd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for hdr in ("hsvd.h", "hsvd_debug.h"):
        with open(os.path.join(ROOT, "include", hdr)) as f:
            txt = f.read()
        names += re.findall(r"^(?:hsvd_status|const char\*)\s+(hsvd_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = H.lib()
    declared = _declared()
    assert len(declared) >= 11
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(H.EXPORTED) == declared


def test_default_options():
    o = H.default_options()
    assert (o.precision, o.rule, o.oversample, o.power_steps, o.refine_steps, o.max_sweeps,
            o.seed, o.refine_eps) == (0, 0, 14, -1, 0, 40, 0, 0.0)


@pytest.mark.parametrize("args", [
    (0, 10, 1, 1, 1, 0.0), (10, 0, 1, 1, 1, 0.0), (10, 10, 0, 1, 1, 0.0),
    (10, 10, 11, 1, 1, 0.0), (10, 10, 1, 0, 1, 0.0), (10, 10, 1, 11, 1, 0.0),
    (10, 10, 1, 1, 0, 0.0), (10, 10, 1, 1, 11, 0.0), (10, 12, 1, 1, 11, 0.0),
    (10, 10, 1, 1, 1, -0.1), (10, 10, 1, 1, 1, 1.0), (10, 10, 1, 1, 1, float("nan")),
])
def test_plan_rejects_bad_arguments(args):
    lib = H.lib()
    h = ctypes.c_void_p(1234)
    st = lib.hsvd_plan(ctypes.byref(h), *args)
    assert st == 1
    assert h.value is None
    assert lib.hsvd_last_error().decode()


def test_plan_rejects_bad_options_and_unsupported_rank():
    lib = H.lib()
    h = ctypes.c_void_p()
    o = H.default_options()
    o.precision = 7
    assert lib.hsvd_plan_ex(ctypes.byref(h), 100, 100, 2, 2, 5, 0.0, ctypes.byref(o)) == 1
    o = H.default_options()
    o.max_sweeps = 0
    assert lib.hsvd_plan_ex(ctypes.byref(h), 100, 100, 2, 2, 5, 0.0, ctypes.byref(o)) == 1
    for bad in (-2, 65):
        o = H.default_options()
        o.power_steps = bad
        assert lib.hsvd_plan_ex(ctypes.byref(h), 100, 100, 2, 2, 5, 0.0, ctypes.byref(o)) == 1
    for bad in (-1e-3, float("nan")):
        o = H.default_options()
        o.refine_steps, o.refine_eps = 3, bad
        assert lib.hsvd_plan_ex(ctypes.byref(h), 100, 100, 2, 2, 5, 0.0, ctypes.byref(o)) == 1
        assert "refine_eps" in lib.hsvd_last_error().decode()
    assert lib.hsvd_plan(ctypes.byref(h), 1000, 1000, 2, 2, 81, 0.0) == 6
    assert "k > 80" in lib.hsvd_last_error().decode()
    assert lib.hsvd_plan(None, 100, 100, 2, 2, 5, 0.0) == 1


def test_null_handles():
    lib = H.lib()
    assert lib.hsvd_destroy(None) == 0
    assert lib.hsvd_execute(None, None, None, None, None, None) == 1
    r = ctypes.c_int32()
    assert lib.hsvd_get_rank(None, ctypes.byref(r)) == 1
    assert lib.hsvd_get_status(None, None) == 1
    assert lib.hsvd_debug_jacobi(None, 1, 4, None, None, None, 10, 0, None, None) == 1
    assert lib.hsvd_debug_tsqr(None, 1, 4, 4, None, None, None) == 1
    assert lib.hsvd_debug_cholqr(None, 1, 4, 4, None, None, None, None) == 1
    assert lib.hsvd_get_refine_iterations(None, ctypes.byref(r)) == 1


@pytest.mark.parametrize("shape", [
    (512, 512, 2, 2, 20, {}),
    (8192, 8192, 8, 8, 50, {"precision": 1}),
    (1000, 900, 3, 4, 20, {}),
    (1000, 900, 3, 4, 20, {"power_steps": 0}),
    (1000, 900, 3, 4, 20, {"power_steps": 2, "refine_steps": 2}),
    (1000, 900, 3, 4, 20, {"power_steps": -1, "rule": 1}),
    (8192, 8192, 8, 8, 50, {"power_steps": -1}),
    (1000, 900, 3, 4, 20, {"power_steps": -1, "refine_steps": 3, "refine_eps": 1e-4}),
    (777, 333, 5, 3, 17, {"rule": 1}),
    (300, 200, 1, 1, 7, {}),
    (10, 7, 10, 7, 1, {}),
    (16384, 16384, 16, 16, 64, {"precision": 1}),
    (2049, 4097, 3, 9, 64, {"oversample": 40}),
    (8192, 8192, 8, 8, 50, {"precision": 2}),
    (1000, 900, 3, 4, 20, {"precision": 2, "refine_steps": 1}),
    (1000, 900, 3, 4, 20, {"refine_steps": 4, "refine_eps": 1e-6}),
    (1000, 900, 3, 4, 20, {"precision": 2, "refine_steps": 2, "refine_eps": 1e-3}),
    (1200, 1100, 3, 3, 80, {}),
    (1000, 1300, 2, 3, 72, {"precision": 2, "refine_steps": 1}),
    (16384, 16384, 16, 16, 80, {"precision": 2}),
])
def test_plan_footprint_is_in_bounds(shape):
    """Every task of every launch stays inside the plan's buffers (host-side check)."""
    m, n, p, q, k, opts = shape
    b = H.plan_check(m, n, p, q, k, 0.0, **opts)
    assert b > 0


def _arr(t, v):
    return (t * len(v))(*v)


def test_batched_plan_rejects_bad_arguments():
    lib = H.lib()
    h = ctypes.c_void_p(1234)
    assert lib.hsvd_plan_batched(ctypes.byref(h), 0, None, None, None, None, None, 0.0, None) == 1
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    ms, ns = _arr(i64, [100, 10]), _arr(i64, [100, 50])
    ps, qs, ks = _arr(i32, [2, 20]), _arr(i32, [2, 2]), _arr(i32, [5, 5])
    assert lib.hsvd_plan_batched(ctypes.byref(h), 2, ms, ns, ps, qs, ks, 0.0, None) == 1
    assert "matrix 1" in lib.hsvd_last_error().decode()
    ks = _arr(i32, [5, 81])
    ms, ns = _arr(i64, [100, 100]), _arr(i64, [100, 100])
    assert lib.hsvd_plan_batched(ctypes.byref(h), 2, ms, ns, _arr(i32, [2, 2]), qs, ks, 0.0, None) == 6
    assert lib.hsvd_execute_batched(None, None, None, None, None, None) == 1
    assert lib.hsvd_get_ranks(None, None, 1) == 1


def test_batched_plan_footprint_uneven_batch():
    """The 200-matrix uneven batch (shapes and grids of the uneven workload, ranks
    5..80, so that both the LDS-resident and the wide merge cores run): every task of
    every launch stays inside its buffers."""
    from paper_1710_02812_amd import synth
    rng = np.random.default_rng(3)
    shapes = []
    for _ in range(200):
        m, n = int(rng.integers(256, 4097)), int(rng.integers(256, 4097))
        k = int(rng.integers(5, 81))
        shapes.append((m, n, -(-m // 512), -(-n // 512), k))
    b = H.plan_check_batched(shapes)
    assert b > 0
    b2 = H.plan_check_batched(shapes[:7], precision=2)
    assert b2 > 0
    single = H.plan_check(*shapes[0])
    assert H.plan_check_batched(shapes[:1]) == single
    assert synth is not None


def _build_or_no_device(st, h):
    """Plan construction and validation run on the host; without a GPU the call
    then stops at the device query (status 3)."""
    lib = H.lib()
    assert st in (0, 3), lib.hsvd_last_error()
    if st == 0:
        lib.hsvd_destroy(h)


def test_feature_and_width_plans_build_on_host():
    lib = H.lib()
    h = ctypes.c_void_p()
    _build_or_no_device(lib.hsvd_features_plan(ctypes.byref(h), 512, 768, 2, 3, 0, 0), h)
    _build_or_no_device(lib.hsvd_features_plan(ctypes.byref(h), 1000, 333, 4, 3, 1, 5), h)
    assert lib.hsvd_features_plan(ctypes.byref(h), 512, 768, 2, 3, 2, 0) == 1
    widths = _arr(ctypes.c_int32, [8, 16, 24, 64, 80, 8])
    o = H.default_options()
    o.rule = 1
    _build_or_no_device(lib.hsvd_plan_widths(ctypes.byref(h), 512, 768, 2, 3, 40, 1e-3, ctypes.byref(o),
                                             widths), h)
    bad = _arr(ctypes.c_int32, [8, 16, 24, 64, 81, 8])
    assert lib.hsvd_plan_widths(ctypes.byref(h), 512, 768, 2, 3, 40, 1e-3, ctypes.byref(o), bad) == 1
    assert lib.hsvd_plan_widths(ctypes.byref(h), 512, 768, 2, 3, 40, 1e-3, ctypes.byref(o), None) == 1
