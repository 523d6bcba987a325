"""GPU checks of the FP32 decode on the matrix cores.

Decoding to FP32 runs axis 0 into an FP32 intermediate, then axes 1 and 2
as FP32 MFMA products with FP32 accumulation (tiles of 16 points, control
windows blocked dense).  Error bound, with u = 2^-24: an output is the
axis-0 value rounded once to FP32, summed over at most 16 control rows of
axis 1 and then over at most 32 products of axis 2 (two 16-column tiles),
plus the roundings of the operands, so its error stays below about
(1 + 16 + 32 + 3) u = 3.1e-6 times the same sum taken over absolute values,
B = (|N_0| x |N_1| x |N_2|) |P| (Higham, Accuracy and Stability of Numerical
Algorithms, eq. 3.5 for recursive summation).  Every case is held to 3.2e-6 B
against the oracle's FP64 decode; values (r = 0) must also meet the
mixed-precision bar of 1e-6 of max |f|.

Shapes cover several 16-point tiles with ragged tails on both axes, odd
and even numbers of 16-column control tiles (the loop takes two per trip),
output rows whose length is not a multiple of 4 (scalar stores), degrees 1
to 6, derivative orders up to 3, and the 2-D case (the control grid is read
directly in FP64, no axis-0 pass).
"""
import os

import numpy as np
import pytest

from oracle import lsq, schwarz
from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BOUND = 3.2e-6

CASES = {
    # ntk = 1, m2 = 33 (scalar stores), ragged axis-1 tiles
    "3d-p3-small": lambda: W.small_3d(),
    # ntk = 3, m2 = 72 (4.5 tiles)
    "3d-p4-72": lambda: W.small_3d(npts=(40, 48, 72), sizes=((8, 9), (10, 10), (18, 18)), p=4, overlap=2),
    # ntk = 7 (odd), m2 = 200, m1 = 70
    "3d-p4-ntk7": lambda: W.small_3d(npts=(20, 70, 200), sizes=((5, 5), (12, 12, 11), (34, 33, 33)), p=4,
                                     overlap=2),
    # ntk = 4 (even), m2 = 130 (scalar stores)
    "3d-p2-ntk4": lambda: W.small_3d(npts=(12, 50, 130), sizes=((4, 4), (9, 9, 8), (16, 16, 16, 16)), p=2,
                                     overlap=2),
    "3d-p1": lambda: W.small_3d(npts=(18, 34, 66), sizes=((4, 4), (8, 8), (16, 16)), p=1, overlap=1),
    # 16 points of axis 1 see at most 4 control rows: one K-step in the first product
    "3d-p1-ks1": lambda: W.small_3d(npts=(10, 128, 64), sizes=((4, 4), (8, 8), (8, 8)), p=1, overlap=1),
    "3d-p6": lambda: W.small_3d(npts=(20, 44, 96), sizes=((7, 7), (11, 11), (22, 22)), p=6, overlap=3),
    # m2 / n2 = 8: most output tiles need a single control tile
    "3d-p3-ratio8": lambda: W.small_3d(npts=(16, 64, 256), sizes=((4, 4), (8, 8), (16, 16)), p=3, overlap=2),
    "2d-p3": lambda: W.Workload("2d-small", (97, 71), 3, [[9, 10, 9], [8, 9]], 2, jump_tol=1e-8, seed=7),
}

DERIVS = {2: [(0, 0), (1, 0), (0, 2), (2, 3)], 3: [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 3, 3)]}


def _setup(w):
    S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
    P = np.random.default_rng(11 + w.degree).standard_normal(w.nctrl)
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "fp64")
    enc.set_ctrl(torch.from_numpy(P).cuda())
    return S, P, enc


def _abs_bound(S, P, der):
    mats = []
    for a, ax in enumerate(S.plan.axes):
        C = S.colls[a] if der[a] == 0 else ax.coll(ax.u, der[a])
        mats.append(np.abs(C))
    return lsq.tensor_apply(mats, np.abs(P))


def _decode32(enc, der, vector):
    if vector:
        os.environ["MFA_VECTOR_DECODE"] = "1"
    try:
        f = enc.decode(dtype=torch.float32, deriv=der)
        torch.cuda.synchronize()
    finally:
        os.environ.pop("MFA_VECTOR_DECODE", None)
    return f.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_decode_within_rounding_bound(name):
    w = CASES[name]()
    print(f"decode fp32 {name}: npts={w.npts} p={w.degree} nctrl={w.nctrl}", flush=True)
    S, P, enc = _setup(w)
    try:
        for der in DERIVS[w.dim]:
            der = tuple(min(r, w.degree) for r in der)   # orders above p are rejected
            ref = schwarz.decode(S, P, der)
            B = _abs_bound(S, P, der)
            got = _decode32(enc, der, vector=False)
            err = np.abs(got - ref)
            assert np.all(err <= BOUND * B + 1e-300), (name, der, float(np.max(err / (B + 1e-300))))
            if not any(der):
                assert np.max(err) <= 1e-6 * np.max(np.abs(ref)), (name, float(np.max(err)))
            vec = _decode32(enc, der, vector=True)
            assert np.all(np.abs(vec - ref) <= BOUND * B + 1e-300), (name, der)
    finally:
        enc.close()


def test_fp32_decode_takes_the_matrix_core_path():
    """On a shape the matrix-core kernel accepts, the FP32 decode is not the
    vector kernels' result bit for bit (different summation order), while
    the FP64 decode stays on the vector kernels (bitwise equal either way)."""
    w = CASES["3d-p4-ntk7"]()
    _, _, enc = _setup(w)
    try:
        mf = _decode32(enc, (0, 0, 0), vector=False)
        vf = _decode32(enc, (0, 0, 0), vector=True)
        assert not np.array_equal(mf, vf)
        d1 = enc.decode().cpu().numpy()
        os.environ["MFA_VECTOR_DECODE"] = "1"
        try:
            d2 = enc.decode().cpu().numpy()
        finally:
            os.environ.pop("MFA_VECTOR_DECODE", None)
        assert np.array_equal(d1, d2)
    finally:
        enc.close()


def test_fp32_decode_repeatable():
    """Two decodes of the same model are bitwise equal (the tables are
    rebuilt per call into the same scratch)."""
    w = CASES["3d-p4-72"]()
    _, _, enc = _setup(w)
    try:
        a = _decode32(enc, (0, 1, 0), vector=False)
        b = _decode32(enc, (0, 1, 0), vector=False)
        assert np.array_equal(a, b)
    finally:
        enc.close()
