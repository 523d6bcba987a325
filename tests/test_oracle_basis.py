"""Pins for the oracle's B-spline basis against closed forms, SciPy and calculus.

Section 2.1 (eq. nurbs-basis, W = 1) and Section 2.2 (clamped global ends,
partition of unity).  SciPy's BSpline is an independent implementation used
here as a black box.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline

CASES = [(10, 1, 37), (12, 2, 50), (20, 3, 77), (80, 3, 2000), (17, 4, 61), (9, 5, 40),
         (7, 6, 23)]


@pytest.mark.parametrize("n,p,m", CASES)
def test_partition_of_unity_and_support(n, p, m):
    t = bspline.clamped_uniform_knots(n, p)
    u = bspline.params(m)
    C = bspline.collocation(t, n, p, u)
    assert np.max(np.abs(C.sum(axis=1) - 1.0)) < 1e-14
    assert C.min() >= -1e-15
    nnz = (np.abs(C) > 0).sum(axis=1)
    assert nnz.max() <= p + 1
    span = bspline.find_span(t, n, p, u)
    for i in range(m):
        nz = np.nonzero(C[i])[0]
        assert nz.min() >= span[i] - p and nz.max() <= span[i]


@pytest.mark.parametrize("n,p,m", CASES)
def test_matches_scipy_design_matrix(n, p, m):
    t = bspline.clamped_uniform_knots(n, p)
    u = bspline.params(m)
    C = bspline.collocation(t, n, p, u)
    ref = BSpline.design_matrix(u, t, p).toarray()
    assert np.max(np.abs(C - ref)) < 1e-13


def test_uniform_cubic_closed_form():
    n, p = 30, 3
    t = bspline.clamped_uniform_knots(n, p)
    h = 1.0 / (n - p)
    rng = np.random.default_rng(0)
    for s in range(2 * p, n - p - 1):
        loc = rng.uniform(0, 1, 7)
        u = t[s] + loc * h
        C = bspline.collocation(t, n, p, u)
        want = np.stack([(1 - loc) ** 3 / 6, (3 * loc ** 3 - 6 * loc ** 2 + 4) / 6,
                         (-3 * loc ** 3 + 3 * loc ** 2 + 3 * loc + 1) / 6, loc ** 3 / 6], axis=1)
        assert np.max(np.abs(C[:, s - 3:s + 1] - want)) < 1e-13


@pytest.mark.parametrize("n,p,m", CASES)
def test_derivatives_match_scipy(n, p, m):
    t = bspline.clamped_uniform_knots(n, p)
    u = bspline.params(m)
    # move off the knots so that order-p derivatives are unambiguous
    uo = np.clip(u + 0.123 / (m * (n - p)), 0, 1 - 1e-12)
    for r in range(0, p + 1):
        C = bspline.collocation(t, n, p, uo, r)
        for j in range(0, n, max(1, n // 7)):
            c = np.zeros(n)
            c[j] = 1.0
            ref = BSpline(t, c, p).derivative(r)(uo) if r else BSpline(t, c, p)(uo)
            scale = max(1.0, np.max(np.abs(ref)))
            assert np.max(np.abs(C[:, j] - ref)) < 1e-11 * scale


def test_derivatives_finite_difference():
    n, p = 15, 4
    t = bspline.clamped_uniform_knots(n, p)
    rng = np.random.default_rng(1)
    u = rng.uniform(0.05, 0.95, 40)
    P = rng.standard_normal(n)
    h = 1e-5
    for r in range(1, p):
        d = bspline.collocation(t, n, p, u, r) @ P
        lo = bspline.collocation(t, n, p, u - h, r - 1) @ P
        hi = bspline.collocation(t, n, p, u + h, r - 1) @ P
        fd = (hi - lo) / (2 * h)
        assert np.max(np.abs(d - fd)) < 1e-4 * max(1.0, np.max(np.abs(d)))


@pytest.mark.parametrize("n,p", [(10, 1), (12, 2), (20, 3), (17, 4)])
def test_marsden_linear_reproduction(n, p):
    """sum_k xi_k N_k(u) = u with xi the Greville abscissae."""
    t = bspline.clamped_uniform_knots(n, p)
    u = bspline.params(101)
    xi = bspline.greville(t, n, p)
    assert np.max(np.abs(bspline.collocation(t, n, p, u) @ xi - u)) < 1e-14
    xf = np.array([float(bspline.greville_fraction(n, p, k)) for k in range(n)])
    assert np.max(np.abs(xf - xi)) < 1e-15


@pytest.mark.parametrize("n,p", [(10, 2), (20, 3), (17, 4), (12, 5)])
def test_derivative_coefficients_are_the_derivative_spline(n, p):
    t = bspline.clamped_uniform_knots(n, p)
    rng = np.random.default_rng(2)
    P = rng.standard_normal(n)
    u = rng.uniform(0, 1, 200)
    for r in range(0, p):
        D = bspline.derivative_coefficients(P, t, p, r)
        spl = BSpline(t[r:len(t) - r], D, p - r)
        ref = BSpline(t, P, p).derivative(r)(u) if r else BSpline(t, P, p)(u)
        assert np.max(np.abs(spl(u) - ref)) < 1e-10 * max(1, np.max(np.abs(ref)))
        # convex hull: the coefficients bound the derivative
        assert np.max(np.abs(ref)) <= np.max(np.abs(D)) * (1 + 1e-12)


def test_derivative_coefficients_of_linear():
    n, p = 14, 3
    t = bspline.clamped_uniform_knots(n, p)
    xi = bspline.greville(t, n, p)
    D1 = bspline.derivative_coefficients(xi, t, p, 1)
    assert np.max(np.abs(D1 - 1.0)) < 1e-13
    D2 = bspline.derivative_coefficients(xi, t, p, 2)
    assert np.max(np.abs(D2)) < 1e-11


def test_span_rule_right_continuous():
    n, p = 9, 2
    t = bspline.clamped_uniform_knots(n, p)
    s = bspline.find_span(t, n, p, np.array([0.0, t[4], 1.0]))
    assert list(s) == [p, 4, n - 1]


def test_spectral_field_fft_route_equals_mode_sum():
    from paper_2210_06528_amd import workloads as W
    for shape, kmax in [((24, 20, 18), 5), ((30, 26), 6)]:
        f = W.field_spectral(shape, nmodes=40, kmax=kmax, seed=3, dtype=np.float64)
        g = W.field_spectral_direct(shape, nmodes=40, kmax=kmax, seed=3)
        assert np.max(np.abs(f - g)) < 1e-12


def test_separable_spectral_field_equals_fft_route():
    """The serving loop's device generator (torch, here on the CPU) evaluates
    the same Fourier sum as the FFT route used for the named workloads."""
    import torch
    from paper_2210_06528_amd import workloads as W
    from paper_2210_06528_amd.serve import spectral_field_torch
    for shape, kmax in [((40, 36, 30), 6), ((50, 44), 8), ((33, 65, 48), 4)]:
        f = spectral_field_torch(shape, kmax, seed=7, device="cpu").numpy()
        g = W.field_spectral(shape, kmax=kmax, seed=7, dtype=np.float32)
        assert np.max(np.abs(f - g)) < 2e-6
