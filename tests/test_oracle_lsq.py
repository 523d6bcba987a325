"""Pins for the oracle's normal equations, banded Cholesky and separable LSQ.

Section 2.1 (eq. minimization-problem) and Section 2.3.1 (Cholesky on the
normal equations).  LAPACK (through SciPy/NumPy) and brute-force dense least
squares on the Kronecker-product matrix are the independent references.
"""
import numpy as np
import pytest
from scipy.linalg import cholesky_banded

from oracle import bspline, lsq


def _coll(n, p, m):
    t = bspline.clamped_uniform_knots(n, p)
    return bspline.collocation(t, n, p, bspline.params(m))


@pytest.mark.parametrize("n,p,m", [(10, 1, 30), (16, 2, 40), (25, 3, 90), (19, 4, 60)])
def test_gram_band_is_dense_gram(n, p, m):
    C = _coll(n, p, m)
    band = lsq.gram_band(C, p)
    assert np.array_equal(lsq.band_to_dense(band), np.tril(C.T @ C) + np.tril(C.T @ C, -1).T)
    # the Gram matrix of degree-p B-splines has half-bandwidth p
    G = C.T @ C
    assert np.all(np.abs(np.triu(G, p + 1)) == 0)


@pytest.mark.parametrize("n,p,m", [(10, 1, 30), (16, 2, 40), (25, 3, 90), (19, 4, 60)])
def test_cholesky_band_matches_lapack(n, p, m):
    band = lsq.gram_band(_coll(n, p, m), p)
    L = lsq.cholesky_band(band)
    ref = cholesky_banded(band, lower=True)
    assert np.max(np.abs(L - ref)) < 1e-13 * np.max(np.abs(ref))
    Ld = np.zeros((n, n))
    for t in range(p + 1):
        for k in range(n - t):
            Ld[k + t, k] = L[t, k]
    assert np.max(np.abs(Ld @ Ld.T - lsq.band_to_dense(band))) < 1e-13


def test_cholesky_rejects_singular():
    # fewer data points than control points in a span: singular normal matrix
    n, p = 12, 3
    t = bspline.clamped_uniform_knots(n, p)
    C = bspline.collocation(t, n, p, np.linspace(0, 0.3, 20))
    with pytest.raises(np.linalg.LinAlgError):
        lsq.cholesky_band(lsq.gram_band(C, p))


def test_band_solve_matches_numpy():
    n, p, m = 21, 3, 70
    band = lsq.gram_band(_coll(n, p, m), p)
    L = lsq.cholesky_band(band)
    rng = np.random.default_rng(0)
    B = rng.standard_normal((n, 4, 3))
    X = lsq.solve_band_cholesky(L, B, axis=0)
    ref = np.linalg.solve(lsq.band_to_dense(band), B.reshape(n, -1)).reshape(B.shape)
    assert np.max(np.abs(X - ref)) < 1e-12 * np.max(np.abs(ref))
    X1 = lsq.solve_band_cholesky(L, np.moveaxis(B, 0, 1), axis=1)
    assert np.max(np.abs(np.moveaxis(X1, 1, 0) - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_separable_lsq_is_dense_lstsq(p):
    """Brute force on a tiny 3-D grid: lstsq on the full Kronecker product."""
    npts, nctrl = (17, 13, 11), (7, 6, 5)
    colls = [_coll(n, p, m) for n, m in zip(nctrl, npts)]
    rng = np.random.default_rng(p)
    Q = rng.standard_normal(npts)
    P = lsq.separable_lsq(Q, colls, p)
    K = np.kron(np.kron(colls[0], colls[1]), colls[2])
    ref, *_ = np.linalg.lstsq(K, Q.ravel(), rcond=None)
    assert np.max(np.abs(P.ravel() - ref)) < 1e-10 * np.max(np.abs(ref))


def test_tensor_apply_is_kron():
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((4, 3)), rng.standard_normal((5, 2)), rng.standard_normal((2, 6))]
    X = rng.standard_normal((3, 2, 6))
    Y = lsq.tensor_apply(mats, X)
    K = np.kron(np.kron(mats[0], mats[1]), mats[2])
    assert np.allclose(Y.ravel(), K @ X.ravel(), rtol=1e-13, atol=1e-13)
