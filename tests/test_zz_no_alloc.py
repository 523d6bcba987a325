"""mfa_create_noalloc: a handle whose workspace is the library's own device
array gives the same setup tables, sweeps and decode as mfa_create with a
caller workspace, on two problems in a row (the second smaller, so the array
still holds the first one's contents), and an older no-allocation handle is
refused once a newer one has claimed the array."""
import numpy as np
import pytest

from oracle import schwarz
from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem_large():
    # 3-D, p = 4, uneven blocks, split-BF16 correction (n2 = 22 takes the
    # fused axis-2/axis-1 pass)
    w = W.small_3d(npts=(120, 100, 90), sizes=((12, 13, 11), (10, 12, 11), (11, 11)), p=4,
                   overlap=2, precision="mixed_bf16", seed=11)
    w.extra["kmax"] = 8
    return w


def _problem_small():
    w = W.Workload("2d-small", (97, 71), 3, [[9, 10, 9], [8, 9]], 2, jump_tol=1e-8, seed=3)
    w.extra["kmax"] = 6
    return w


def _run(w, noalloc, q, sweeps, tol):
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, w.precision, noalloc=noalloc)
    st = enc.encode(q, sweeps, tol, 0 if tol > 0 else 1)
    P = enc.get_ctrl().cpu().numpy()
    f = enc.decode(dtype=torch.float64).cpu().numpy()
    d1 = enc.decode(dtype=torch.float32, deriv=[1] + [0] * (len(w.npts) - 1)).cpu().numpy()
    chol = enc.inspect("chol", axis=0, block=1)
    torch.cuda.synchronize()
    return enc, st, P, f, d1, chol


def test_noalloc_matches_workspace_handle_twice():
    print("noalloc: large 3-D mixed_bf16 problem, then a smaller 2-D FP64 one", flush=True)
    wl = _problem_large()
    ql = torch.from_numpy(W.field_spectral(wl.npts, kmax=8, seed=wl.seed, dtype=np.float64)).cuda()
    ws = _lib.workspace_size(wl.npts, wl.degree, wl.sizes, wl.overlap, wl.precision)
    assert ws <= _lib.NOALLOC_MAX_BYTES
    ref = _run(wl, False, ql, 200, 1e-8)
    na = _run(wl, True, ql, 200, 1e-8)
    assert ref[1]["converged"] and na[1]["converged"]
    assert ref[1]["sweep"] == na[1]["sweep"]
    for a, b in zip(ref[2:], na[2:]):
        np.testing.assert_array_equal(a, b)
    ref[0].close()

    # second call, smaller input: the array still holds the first problem
    ws_small = _problem_small()
    Q = W.field_spectral(ws_small.npts, kmax=6, seed=ws_small.seed, dtype=np.float64)
    qs = torch.from_numpy(Q).cuda()
    ref2 = _run(ws_small, False, qs, 6, 0.0)
    na2 = _run(ws_small, True, qs, 6, 0.0)
    for a, b in zip(ref2[2:], na2[2:]):
        np.testing.assert_array_equal(a, b)
    # and both agree with the oracle's literal sweeps (FP64 parity bar)
    S = schwarz.setup(schwarz.make_plan(ws_small.npts, ws_small.degree, ws_small.sizes,
                                        ws_small.overlap))
    Po, _ = schwarz.encode(S, Q, 6)
    assert np.max(np.abs(na2[2] - Po)) <= 1e-10 * np.max(np.abs(Po))

    # the first no-allocation handle lost the array to the second
    with pytest.raises(_lib.MfaError) as ei:
        na[0].get_ctrl()
    assert ei.value.status == _lib.MFA_EINVAL and "newer handle" in str(ei.value)
    na[0].close()
    # the current one still works
    P2 = na2[0].get_ctrl().cpu().numpy()
    np.testing.assert_array_equal(P2, na2[2])
    na2[0].close()
    ref2[0].close()


def test_noalloc_rejects_problem_beyond_the_array():
    w = W.cfg_3d_mixed()   # 1.5 GB of workspace
    with pytest.raises(_lib.MfaError) as ei:
        _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, w.precision, noalloc=True)
    assert ei.value.status == _lib.MFA_ENOMEM
