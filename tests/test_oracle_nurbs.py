"""Pins of the oracle's rational (NURBS) basis and of the weighted fit.

Section 2.1 (eq. nurbs-basis) defines R_i = N_i W_i / sum_j N_j W_j; the
conclusions extend the method to W != 1.  None of these checks uses the
oracle to check itself:
  * all weights equal (1 or any constant) give the B-spline basis;
  * R_0 against SciPy's B-spline design matrix weighted and normalised;
  * partition of unity, and derivative rows summing to zero;
  * the rational quadratic quarter circle (weights 1, sqrt(2)/2, 1): every
    point lies on the unit circle, the first derivative is tangent to it and
    the second satisfies the differentiated identity (pins r = 0, 1, 2);
  * derivative rows against central finite differences of R;
  * a weighted spline of the same space is reproduced exactly by the
    single-domain fit and by the converged Schwarz sweeps, and the fit equals
    brute-force dense least squares on the Kronecker product.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline, lsq, schwarz

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _knots(n, p):
    return bspline.clamped_uniform_knots(n, p)


@pytest.mark.parametrize("p,n", [(2, 7), (3, 11), (4, 9)])
def test_constant_weights_give_the_bspline_basis(p, n):
    t = _knots(n, p)
    u = np.linspace(0.0, 1.0, 97)
    for c in (1.0, 3.7):
        for r in range(p + 1):
            R = bspline.rational_collocation(t, n, p, u, np.full(n, c), r)
            C = bspline.collocation(t, n, p, u, r)
            assert np.max(np.abs(R - C)) < 1e-12 * max(1.0, np.max(np.abs(C)))


def test_values_against_scipy_design_matrix():
    rng = np.random.default_rng(0)
    p, n = 3, 12
    t = _knots(n, p)
    u = rng.random(200)
    w = rng.uniform(0.3, 3.0, n)
    N = BSpline.design_matrix(u, t, p).toarray()
    ref = N * w[None, :] / (N @ w)[:, None]
    assert np.max(np.abs(bspline.rational_collocation(t, n, p, u, w) - ref)) < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4])
def test_partition_of_unity_and_derivative_row_sums(p):
    rng = np.random.default_rng(p)
    n = 10
    t = _knots(n, p)
    u = np.linspace(0.0, 1.0, 151)
    w = rng.uniform(0.2, 5.0, n)
    assert np.max(np.abs(bspline.rational_collocation(t, n, p, u, w).sum(axis=1) - 1.0)) < 1e-14
    for r in range(1, p + 1):
        D = bspline.rational_collocation(t, n, p, u, w, r)
        assert np.max(np.abs(D.sum(axis=1))) < 1e-9 * max(1.0, np.max(np.abs(D)))


def test_quarter_circle():
    """Rational quadratic Bezier arc with control points (1,0), (1,1), (0,1)
    and weights (1, sqrt(2)/2, 1) is the quarter of the unit circle."""
    p, n = 2, 3
    t = _knots(n, p)
    w = np.array([1.0, np.sqrt(0.5), 1.0])
    Px, Py = np.array([1.0, 1.0, 0.0]), np.array([0.0, 1.0, 1.0])
    u = np.linspace(0.0, 1.0, 401)
    R = [bspline.rational_collocation(t, n, p, u, w, r) for r in range(3)]
    x, y = [Rr @ Px for Rr in R], [Rr @ Py for Rr in R]
    assert np.max(np.abs(x[0] ** 2 + y[0] ** 2 - 1.0)) < 1e-14
    # |C|^2 = 1  =>  C . C' = 0  and  C . C'' + |C'|^2 = 0
    assert np.max(np.abs(x[0] * x[1] + y[0] * y[1])) < 1e-13
    assert np.max(np.abs(x[0] * x[2] + y[0] * y[2] + x[1] ** 2 + y[1] ** 2)) < 1e-12
    # a weight of 1 in the middle would give the parabola, off the circle
    Rb = bspline.rational_collocation(t, n, p, u, np.ones(3))
    assert np.max(np.abs((Rb @ Px) ** 2 + (Rb @ Py) ** 2 - 1.0)) > 0.1


@pytest.mark.parametrize("r", [1, 2, 3])
def test_derivatives_against_finite_differences(r):
    rng = np.random.default_rng(4)
    p, n = 4, 9
    t = _knots(n, p)
    w = rng.uniform(0.5, 2.0, n)
    # points inside spans (away from knots, where derivatives are smooth)
    u = (np.arange(n - p) + 0.37) / (n - p)
    h = 1e-3 if r < 3 else 3e-4    # truncation error O(h^2) of each stencil
    f = lambda x: bspline.rational_collocation(t, n, p, x, w)
    if r == 1:
        fd = (f(u + h) - f(u - h)) / (2 * h)
    elif r == 2:
        fd = (f(u + h) - 2 * f(u) + f(u - h)) / h ** 2
    else:
        fd = (f(u + 2 * h) - 2 * f(u + h) + 2 * f(u - h) - f(u - 2 * h)) / (2 * h ** 3)
    D = bspline.rational_collocation(t, n, p, u, w, r)
    assert np.max(np.abs(D - fd)) < 1e-4 * max(1.0, np.max(np.abs(D)))


def _weighted_case(dim, p=3, seed=1):
    rng = np.random.default_rng(seed)
    if dim == 1:
        npts, sizes = (300,), [[12, 13, 11]]
    else:
        npts, sizes = (61, 53), [[9, 8], [8, 9]]
    ws = [rng.uniform(0.4, 2.5, sum(s)) for s in sizes]
    plan = schwarz.make_plan(npts, p, sizes, 2, weights=ws)
    return plan, ws, rng


@pytest.mark.parametrize("dim", [1, 2])
def test_weighted_spline_reproduced_exactly(dim):
    plan, ws, rng = _weighted_case(dim)
    S = schwarz.setup(plan)
    P = rng.standard_normal(plan.nctrl)
    Q = schwarz.decode(S, P)
    Pd = schwarz.global_direct(S, Q)
    assert np.max(np.abs(Pd - P)) < 1e-10 * np.max(np.abs(P))
    Ps, hist = schwarz.encode(S, Q, 200, jump_tol=1e-12)
    assert np.max(np.abs(Ps - P)) < 1e-8 * np.max(np.abs(P))
    # the weights matter: the unweighted fit of the same data is not exact
    plan_b = schwarz.make_plan(tuple(ax.m for ax in plan.axes), plan.p,
                               [[b.c1 - b.c0 for b in ax.blocks] for ax in plan.axes], 2)
    Pb = schwarz.global_direct(schwarz.setup(plan_b), Q)
    assert np.max(np.abs(Pb - P)) > 1e-3


def test_weighted_fit_equals_dense_least_squares():
    plan, ws, rng = _weighted_case(2, seed=3)
    S = schwarz.setup(plan)
    Q = rng.standard_normal(tuple(ax.m for ax in plan.axes))
    K = np.kron(S.colls[0], S.colls[1])
    ref = np.linalg.lstsq(K, Q.ravel(), rcond=None)[0].reshape(plan.nctrl)
    got = schwarz.global_direct(S, Q)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_invalid_weights_rejected():
    with pytest.raises(ValueError):
        schwarz.make_plan((100,), 3, [[20, 20]], 2, weights=[np.full(40, -1.0)])
    with pytest.raises(ValueError):
        schwarz.make_plan((100,), 3, [[20, 20]], 2, weights=[np.ones(39)])
