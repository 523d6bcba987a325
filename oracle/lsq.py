"""Least-squares pieces: normal equations, banded Cholesky, separable solves.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1 (eq. minimization-problem) poses the per-subdomain fit as
argmin ||Q - R P||_2; Section 2.3.1 names Cholesky on the normal equations
R^T R P = R^T Q as one direct solver.  On a tensor grid R is the Kronecker
product of one collocation matrix per axis, so R^T R is the Kronecker product
of the per-axis Gram matrices and every solve factors axis by axis.

Banded storage is LAPACK-style lower storage: band[t, k] = A[k+t, k] for
t = 0..p (entries past the matrix end are zero).
"""
import numpy as np


def mode_product(M, X, axis):
    """Multiply tensor X by matrix M along `axis`: Y[..i..] = sum_j M[i, j] X[..j..]."""
    Y = np.tensordot(M, X, axes=([1], [axis]))
    return np.moveaxis(Y, 0, axis)


def tensor_apply(mats, X):
    """Apply one matrix per axis (the Kronecker product of `mats`) to X."""
    for a, M in enumerate(mats):
        X = mode_product(M, X, a)
    return X


def gram_band(C, p):
    """Lower band (p+1, n) of the Gram matrix C^T C of a collocation matrix C."""
    A = C.T @ C
    n = A.shape[0]
    band = np.zeros((p + 1, n))
    for t in range(p + 1):
        for k in range(n - t):
            band[t, k] = A[k + t, k]
    return band


def band_to_dense(band):
    """Symmetric dense matrix from its lower band."""
    w, n = band.shape
    A = np.zeros((n, n))
    for t in range(w):
        for k in range(n - t):
            A[k + t, k] = band[t, k]
            A[k, k + t] = band[t, k]
    return A


def cholesky_band(band):
    """Banded Cholesky A = L L^T from the definition, column by column.

    L_jj = sqrt(A_jj - sum_{k<j} L_jk^2) and
    L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj for j < i <= j+p.
    Returns L in the same lower band storage.  Raises on a non-positive pivot
    (the normal matrix is singular: some basis function has no data point in
    its support).
    """
    w, n = band.shape
    p = w - 1
    L = np.zeros_like(band)

    def Lget(i, j):  # L[i, j] for i >= j
        t = i - j
        return L[t, j] if 0 <= t <= p else 0.0

    def Aget(i, j):
        t = i - j
        return band[t, j] if 0 <= t <= p else 0.0

    for j in range(n):
        s = Aget(j, j) - sum(Lget(j, k) ** 2 for k in range(max(0, j - p), j))
        if not s > 0.0:
            raise np.linalg.LinAlgError("normal matrix is not positive definite")
        L[0, j] = np.sqrt(s)
        for i in range(j + 1, min(n, j + p + 1)):
            s = Aget(i, j) - sum(Lget(i, k) * Lget(j, k)
                                 for k in range(max(0, i - p), j))
            L[i - j, j] = s / L[0, j]
    return L


def solve_band_cholesky(L, B, axis=0):
    """Solve (L L^T) X = B along `axis` by forward then backward substitution."""
    w, n = L.shape
    p = w - 1
    X = np.moveaxis(np.array(B, dtype=np.float64, copy=True), axis, 0)
    # forward: L y = b
    for i in range(n):
        for k in range(max(0, i - p), i):
            X[i] -= L[i - k, k] * X[k]
        X[i] /= L[0, i]
    # backward: L^T x = y
    for i in range(n - 1, -1, -1):
        for k in range(i + 1, min(n, i + p + 1)):
            X[i] -= L[k - i, i] * X[k]
        X[i] /= L[0, i]
    return np.moveaxis(X, 0, axis)


def separable_lsq(Q, colls, p):
    """Least-squares fit of tensor data Q with one collocation matrix per axis.

    Solves the normal equations (kron C_a)^T (kron C_a) P = (kron C_a)^T Q,
    which split into one banded Cholesky solve per axis.
    """
    rhs = tensor_apply([C.T for C in colls], Q)
    for a, C in enumerate(colls):
        L = cholesky_band(gram_band(C, p))
        rhs = solve_band_cholesky(L, rhs, axis=a)
    return rhs
