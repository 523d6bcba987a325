"""GPU checks of the per-class event timing (mfa_set_timing,
mfa_set_timing_every, mfa_kernel_time): which launches get an event pair,
what the count reports, and that timing never changes a result."""
import numpy as np
import pytest

from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup():
    w = W.small_3d()
    q = torch.from_numpy(W.field_spectral(w.npts, kmax=w.extra["kmax"], seed=w.seed,
                                          dtype=np.float64)).cuda()
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "fp64")
    return enc, q


def _steps(enc, q, n):
    for k in range(n):
        enc.step(q if k == 0 else None)


@pytest.mark.parametrize("every,first,expect", [(1, 0, 7), (3, 0, 3), (3, 2, 2), (7, 6, 1), (10, 0, 1),
                                                (10, 7, 0)])
def test_sampled_timing_counts_launches_first_plus_multiples_of_every(every, first, expect):
    """Seven sweeps launch the residual stencil seven times (0..6): every = 1
    times all, (3, 0) launches 0, 3, 6, (3, 2) launches 2 and 5, (7, 6) the
    last, (10, 0) the first and (10, 7) none."""
    enc, q = _setup()
    try:
        enc.set_timing(True, ("resid",), every, first)
        _steps(enc, q, 7)
        ms, n = enc.kernel_time("resid")
        assert n == expect
        assert (ms > 0.0) == (expect > 0)
        # untimed classes report nothing; a read resets the class
        assert enc.kernel_time("decode") == (0.0, 0)
        assert enc.kernel_time("resid") == (0.0, 0)
    finally:
        enc.close()


def test_setting_timing_again_restarts_the_sampling():
    enc, q = _setup()
    try:
        enc.set_timing(True, ("resid",), 4)
        _steps(enc, q, 2)          # launch 0 timed, 1 not
        enc.set_timing(True, ("resid",), 4)
        _steps(enc, q, 5)          # counting restarts: launches 0 and 4 timed
        assert enc.kernel_time("resid")[1] == 2
        enc.set_timing(False)
        _steps(enc, q, 2)
        assert enc.kernel_time("resid") == (0.0, 0)
    finally:
        enc.close()


def test_timing_sample_rejects_bad_strides_and_leaves_results_unchanged():
    enc, q = _setup()
    ref, _ = _setup()
    try:
        for every, first in ((0, 0), (3, 3), (3, -1)):
            with pytest.raises(_lib.MfaError) as ei:
                enc.set_timing(True, None, every, first)
            assert ei.value.status == _lib.MFA_EINVAL
        enc.set_timing(True, None, 2, 1)
        _steps(enc, q, 3)
        _steps(ref, q, 3)
        assert np.array_equal(enc.get_ctrl().cpu().numpy(), ref.get_ctrl().cpu().numpy())
    finally:
        enc.close()
        ref.close()
