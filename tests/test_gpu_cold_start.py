"""GPU checks that an encode without a warm start begins from P = 0 whatever
the handle did before: a new handle (whose zeros mfa_create wrote), a
second encode on the same handle, and an encode after single sweeps must
all give the same control points bit for bit."""
import numpy as np
import pytest

from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", ["fp64", "mixed_bf16"])
def test_cold_encode_is_independent_of_the_handle_history(precision):
    w = W.small_3d(npts=(40, 48, 72), sizes=((8, 9), (10, 10), (18, 18)), p=4)
    q = torch.from_numpy(W.field_spectral(w.npts, kmax=w.extra["kmax"], seed=w.seed,
                                          dtype=np.float64)).cuda()
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, precision)
    try:
        enc.encode(q, 8, 0.0, 1)
        first = enc.get_ctrl().cpu().numpy()
        enc.encode(q, 8, 0.0, 1)
        assert np.array_equal(enc.get_ctrl().cpu().numpy(), first)
        enc.step(q)
        enc.step()
        enc.encode(q, 8, 0.0, 1)
        assert np.array_equal(enc.get_ctrl().cpu().numpy(), first)
        enc.recreate()
        enc.encode(q, 8, 0.0, 1)
        assert np.array_equal(enc.get_ctrl().cpu().numpy(), first)
    finally:
        enc.close()
