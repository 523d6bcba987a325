"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and the host planner validates problems (no device calls)."""
import os
import re

import numpy as np
import pytest

from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mfa.h")).read()
    return sorted(set(re.findall(r"\b(mfa_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2210_06528_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_size_for_named_workloads(lib):
    for w in [W.cfg_1d(), W.cfg_2d(), W.cfg_3d_batched(), W.cfg_3d_mixed()]:
        b = _lib.workspace_size(w.npts, w.degree, w.sizes, w.overlap, "fp64")
        # at least the N^T Q, control point and residual arrays in float64
        assert b >= 3 * 8 * int(np.prod(w.nctrl))


@pytest.mark.parametrize("kwargs,msg", [
    (dict(npts=(100,), degree=3, sizes=[[10, 10]], overlap=0), "overlap"),
    (dict(npts=(100,), degree=4, sizes=[[10, 10]], overlap=1), "overlap"),
    (dict(npts=(100,), degree=3, sizes=[[3, 17]], overlap=1), "owned block"),
    (dict(npts=(10,), degree=3, sizes=[[8, 8]], overlap=1), "fewer data points"),
    (dict(npts=(100,), degree=0, sizes=[[10, 10]], overlap=1), "degree"),
    (dict(npts=(100,), degree=9, sizes=[[10, 10]], overlap=1), "degree"),
    (dict(npts=(10, 10, 10, 10), degree=2, sizes=[[5]] * 4, overlap=1), "dim"),
    (dict(npts=(100,), degree=3, sizes=[[2]], overlap=1), "p+1"),
])
def test_invalid_problems_are_rejected(lib, kwargs, msg):
    with pytest.raises(_lib.MfaError) as ei:
        _lib.workspace_size(**kwargs)
    assert ei.value.status == _lib.MFA_EINVAL
    assert msg in str(ei.value)


def test_bad_enum_values_rejected(lib):
    for key in ("precision", "combine", "rhs"):
        kw = dict(npts=(100,), degree=3, sizes=[[20, 20]], overlap=2)
        kw[key] = 7
        with pytest.raises(_lib.MfaError):
            _lib.workspace_size(**kw)


def test_null_pointers_rejected(lib):
    import ctypes
    assert lib.mfa_workspace_size(None, None) == _lib.MFA_EINVAL
    assert b"null" in lib.mfa_last_error()
    assert lib.mfa_create(None, None, 0, None, None) == _lib.MFA_EINVAL
    h = ctypes.c_void_p(0)
    prob, keep = _lib.make_problem((100,), 3, [[20, 20]], 2)
    assert lib.mfa_create(ctypes.byref(prob), None, 0, None, ctypes.byref(h)) == _lib.MFA_EINVAL
    assert lib.mfa_encode(None, None, 0, 1, 0.0, 1, None) == _lib.MFA_EINVAL
    assert lib.mfa_decode(None, None, 0, None) == _lib.MFA_EINVAL
    lib.mfa_destroy(None)


def test_workspace_grows_with_problem(lib):
    a = _lib.workspace_size((200, 200), 3, [[25, 25]] * 2, 2)
    b = _lib.workspace_size((400, 400), 3, [[50, 50]] * 2, 2)
    assert b > 3 * a


def test_noalloc_rejects_oversized_problem_before_device_work(lib):
    import ctypes
    w = W.cfg_3d_mixed()
    assert _lib.workspace_size(w.npts, w.degree, w.sizes, w.overlap, "mixed_bf16") > \
        _lib.NOALLOC_MAX_BYTES
    prob, keep = _lib.make_problem(w.npts, w.degree, w.sizes, w.overlap, "mixed_bf16")
    h = ctypes.c_void_p(0)
    assert lib.mfa_create_noalloc(ctypes.byref(prob), None, ctypes.byref(h)) == _lib.MFA_ENOMEM
    assert b"no-allocation array" in lib.mfa_last_error()
    assert not h.value
    assert lib.mfa_create_noalloc(None, None, None) == _lib.MFA_EINVAL
    bad, keep2 = _lib.make_problem((100,), 3, [[10, 10]], 0)
    assert lib.mfa_create_noalloc(ctypes.byref(bad), None, ctypes.byref(h)) == _lib.MFA_EINVAL


def test_noalloc_array_covers_the_mid_size_workloads(lib):
    # the 256^3 workload and the largest serving request fit the array
    w = W.cfg_3d_batched()
    assert _lib.workspace_size(w.npts, w.degree, w.sizes, w.overlap, "mixed_bf16") <= \
        _lib.NOALLOC_MAX_BYTES


def _unbound_encoder(npts=(6, 5), nctrl=(4, 4)):
    """An Encoder shell on the 'meta' device: argument checks run, nothing
    reaches the library (no handle)."""
    import torch
    enc = _lib.Encoder.__new__(_lib.Encoder)
    enc.torch = torch
    enc.npts, enc.nctrl, enc.dim = tuple(npts), tuple(nctrl), len(npts)
    enc.device = torch.device("meta")
    enc.handle = None
    return enc


@pytest.mark.parametrize("call", ["decode", "decode_points", "set_ctrl"])
def test_binding_rejects_wrong_device_and_dtype(call):
    import torch
    enc = _unbound_encoder()
    meta = dict(device="meta")
    if call == "decode":
        with pytest.raises(TypeError):
            enc.decode(out=torch.empty(enc.npts, dtype=torch.float16, **meta))
        with pytest.raises(TypeError):
            enc.decode(out=torch.empty(enc.npts, dtype=torch.int32, **meta))
        with pytest.raises(ValueError):
            enc.decode(out=torch.empty(enc.npts, dtype=torch.float32))          # host tensor
        with pytest.raises(ValueError):
            enc.decode(out=torch.empty((6, 4), dtype=torch.float32, **meta))    # shape
    elif call == "decode_points":
        u = torch.empty((3, 2), dtype=torch.float64, **meta)
        with pytest.raises(TypeError):
            enc.decode_points(u, out=torch.empty(3, dtype=torch.bfloat16, **meta))
        with pytest.raises(ValueError):
            enc.decode_points(u, out=torch.empty(3, dtype=torch.float64))
        with pytest.raises(ValueError):
            enc.decode_points(torch.empty((3, 2), dtype=torch.float64), dtype=torch.float64)
    else:
        with pytest.raises(ValueError):
            enc.set_ctrl(torch.empty(enc.nctrl, dtype=torch.float64))            # host tensor
        with pytest.raises(ValueError):
            enc.set_ctrl(torch.empty(enc.nctrl, dtype=torch.float32, **meta))


@pytest.mark.parametrize("extent,msg", [([(1.0, 0.0)], "hi < lo"),
                                        ([(0.0, float("inf"))], "not finite"),
                                        ([(float("nan"), 1.0)], "not finite")])
def test_bad_axis_extent_rejected(lib, extent, msg):
    import ctypes
    prob, keep = _lib.make_problem((100,), 3, [[20, 20]], 2, extent=extent)
    out = ctypes.c_size_t(0)
    assert lib.mfa_workspace_size(ctypes.byref(prob), ctypes.byref(out)) == _lib.MFA_EINVAL
    assert msg in lib.mfa_last_error().decode()
    ok, keep2 = _lib.make_problem((100,), 3, [[20, 20]], 2, extent=[(-2.0, 5.0)])
    assert lib.mfa_workspace_size(ctypes.byref(ok), ctypes.byref(out)) == _lib.MFA_OK


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
def test_bad_weights_rejected(lib, bad):
    import ctypes
    w = np.ones(40)
    w[7] = bad
    prob, keep = _lib.make_problem((100,), 3, [[20, 20]], 2, weights=[w])
    out = ctypes.c_size_t(0)
    assert lib.mfa_workspace_size(ctypes.byref(prob), ctypes.byref(out)) == _lib.MFA_EINVAL
    assert b"weight" in lib.mfa_last_error()
    ok, keep2 = _lib.make_problem((100,), 3, [[20, 20]], 2, weights=[np.full(40, 2.0)])
    assert lib.mfa_workspace_size(ctypes.byref(ok), ctypes.byref(out)) == _lib.MFA_OK


def test_variant_ctrl_dims_and_validation(lib):
    from oracle import schwarz, variants
    npts, sizes, p = (61, 47), [[9, 9], [7, 8, 7]], 3
    prob, keep = _lib.make_problem(npts, p, sizes, 2, variant="clamped")
    axes = variants.plan_clamped(npts, p, sizes)
    assert _lib.ctrl_dims_of(prob) == tuple(ax.n for ax in axes)
    prob, keep = _lib.make_problem(npts, p, sizes, 2, variant="decoupled")
    plan = schwarz.make_plan(npts, p, sizes, 2)
    assert _lib.ctrl_dims_of(prob) == tuple(sum(b.F1 - b.F0 for b in ax.blocks) for ax in plan.axes)
    prob, keep = _lib.make_problem(npts, p, sizes, 2)
    assert _lib.ctrl_dims_of(prob) == tuple(sum(s) for s in sizes)
    for kw in (dict(precision="mixed_bf16", variant="clamped"),
               dict(rhs="databox", variant="decoupled"),
               dict(variant=3)):
        with pytest.raises(_lib.MfaError):
            _lib.workspace_size(npts, p, sizes, 2, **kw)
    # a clamped block with fewer data points than control points
    with pytest.raises(_lib.MfaError):
        _lib.workspace_size((20,), 3, [[12, 12]], 2, variant="clamped")
    with pytest.raises(_lib.MfaError):
        _lib.workspace_size((100,), 3, [[20, 20]], 2, variant="clamped", precision="mixed_fp32")
