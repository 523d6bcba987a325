"""B-spline basis on a clamped uniform knot vector, written from the definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.1 (eq. nurbs-basis) and the Cox-de Boor recurrence the
paper cites for values and exact derivatives: plain B-splines (all weights
W = 1), and the rational basis R_i = N_i W_i / sum_j N_j W_j with its
derivatives by the quotient rule (`rational_collocation`).  Knot placement
follows Section 2.2: one knot vector per axis, clamped (p+1 repeated knots)
at the two ends of the global domain and uniform (floating) in the interior,
so a subdomain's knots are a slice of it.

Everything here is float64 and evaluates the recurrence over *all* basis
functions of every degree (dense tables), which is slow but easy to check by
eye.  The span rule, the Greville abscissae and the derivative-coefficient
formula are the textbook ones (de Boor, "A Practical Guide to Splines").
"""
from fractions import Fraction
from math import comb

import numpy as np


def clamped_uniform_knots(n, p):
    """Knots t_0..t_{n+p} for n control points of degree p on [0, 1].

    t_j = clamp((j - p) / (n - p), 0, 1): p+1 copies of 0 and of 1 and n-p
    uniform spans in between (Section 2.2, clamped global ends, floating
    interior knots).
    """
    if n < p + 1:
        raise ValueError("need at least p+1 control points")
    j = np.arange(n + p + 1, dtype=np.float64)
    return np.clip((j - p) / (n - p), 0.0, 1.0)


def params(m):
    """Parameter of each of m uniformly spaced data points: u_i = i / (m-1)."""
    if m < 2:
        raise ValueError("need at least two points per axis")
    return np.arange(m, dtype=np.float64) / (m - 1)


def find_span(t, n, p, u):
    """Right-continuous knot span of each parameter.

    The span of u is the largest s with t_s <= u, restricted to the valid
    range [p, n-1]; u = 1 therefore belongs to the last span n-1.
    """
    u = np.asarray(u, dtype=np.float64)
    s = np.searchsorted(t, u, side="right") - 1
    return np.clip(s, p, n - 1)


def _safe_div(num, den):
    out = np.zeros(np.broadcast(num, den).shape)
    nz = den != 0.0
    np.divide(num, den, out=out, where=nz)
    return out


def basis_tables(t, n, p, u):
    """All B-spline functions of degrees 0..p at the parameters u.

    Returns a list `tab` with tab[k] of shape (len(u), n+p-k): tab[k][i, j] is
    N_{j,k}(u_i).  Degree 0 is the indicator of the span (right-continuous
    rule above), higher degrees follow the Cox-de Boor recurrence

        N_{j,k}(u) = (u - t_j)/(t_{j+k} - t_j) N_{j,k-1}(u)
                   + (t_{j+k+1} - u)/(t_{j+k+1} - t_{j+1}) N_{j+1,k-1}(u)

    with 0/0 read as 0 (repeated knots).
    """
    u = np.asarray(u, dtype=np.float64)
    nfun0 = len(t) - 1
    span = find_span(t, n, p, u)
    tab0 = np.zeros((len(u), nfun0))
    tab0[np.arange(len(u)), span] = 1.0
    tabs = [tab0]
    for k in range(1, p + 1):
        prev = tabs[-1]
        nf = nfun0 - k
        j = np.arange(nf)
        left = _safe_div(u[:, None] - t[j][None, :], (t[j + k] - t[j])[None, :])
        right = _safe_div(t[j + k + 1][None, :] - u[:, None],
                          (t[j + k + 1] - t[j + 1])[None, :])
        tabs.append(left * prev[:, :nf] + right * prev[:, 1:nf + 1])
    return tabs


def collocation(t, n, p, u, r=0):
    """Dense matrix of r-th derivatives: C[i, j] = d^r/du^r N_{j,p}(u_i).

    Derivatives follow the differentiated recurrence

        d/du N_{j,k} = k/(t_{j+k} - t_j) N_{j,k-1} - k/(t_{j+k+1} - t_{j+1}) N_{j+1,k-1}

    applied r times (0/0 read as 0).  For r > p the result is zero.
    """
    tabs = basis_tables(t, n, p, u)
    m = len(np.atleast_1d(u))
    if r > p:
        return np.zeros((m, n))

    def d(r_, k):
        # r_-th derivative of all degree-k functions, shape (m, n+p-k)
        if r_ == 0:
            return tabs[k]
        lower = d(r_ - 1, k - 1)
        nf = len(t) - 1 - k
        j = np.arange(nf)
        a = _safe_div(np.full(nf, float(k)), t[j + k] - t[j])
        b = _safe_div(np.full(nf, float(k)), t[j + k + 1] - t[j + 1])
        return a[None, :] * lower[:, :nf] - b[None, :] * lower[:, 1:nf + 1]

    out = d(r, p)
    return out[:, :n]


def greville(t, n, p):
    """Greville abscissae xi_k = (t_{k+1} + ... + t_{k+p}) / p, k = 0..n-1."""
    return np.array([t[k + 1:k + p + 1].sum() / p for k in range(n)])


def greville_fraction(n, p, k):
    """Greville abscissa xi_k as an exact rational for the clamped uniform knots."""
    tot = Fraction(0)
    for j in range(k + 1, k + p + 1):
        tot += Fraction(min(max(j - p, 0), n - p), n - p)
    return tot / p


def derivative_coefficients(P, t, p, r, axis=0):
    """Control coefficients of the r-th derivative of a spline along one axis.

    For f = sum_k P_k N_{k,p} the derivative is sum_k D_k N_{k+1,p-1} with
    D_k = p (P_{k+1} - P_k) / (t_{k+p+1} - t_{k+1}) on the same knots; applying
    this r times gives the coefficients of d^r f / du^r (degree p-r).
    """
    D = np.moveaxis(np.asarray(P, dtype=np.float64), axis, 0)
    tt = np.asarray(t, dtype=np.float64)
    q = p
    for _ in range(r):
        nn = D.shape[0]
        k = np.arange(nn - 1)
        den = tt[k + q + 1] - tt[k + 1]
        fac = _safe_div(np.full(nn - 1, float(q)), den)
        D = fac.reshape((-1,) + (1,) * (D.ndim - 1)) * (D[1:] - D[:-1])
        tt = tt[1:-1]
        q -= 1
    return np.moveaxis(D, 0, axis)


def rational_collocation(t, n, p, u, w, r=0):
    """Dense matrix of r-th derivatives of the rational basis of eq.
    nurbs-basis: R_j(u) = N_{j,p}(u) w_j / W(u), W(u) = sum_k N_{k,p}(u) w_k.

    With A_j = N_{j,p} w_j (so that A = W R), Leibniz's rule on A = W R gives
    A^(r) = sum_{k=0..r} C(r, k) W^(k) R^(r-k), hence

        R^(r) = ( A^(r) - sum_{k=1..r} C(r, k) W^(k) R^(r-k) ) / W

    computed for r = 0, 1, ... in turn; W^(k) is the row sum of A^(k).
    w = None (or all ones) gives the B-spline collocation.
    """
    if w is None:
        return collocation(t, n, p, u, r)
    w = np.asarray(w, dtype=np.float64)
    if w.shape != (n,) or not np.all(w > 0):
        raise ValueError("weights must be n positive values")
    A = [collocation(t, n, p, u, k) * w[None, :] for k in range(r + 1)]
    Wd = [a.sum(axis=1) for a in A]
    R = []
    for k in range(r + 1):
        acc = A[k].copy()
        for j in range(1, k + 1):
            acc -= comb(k, j) * Wd[j][:, None] * R[k - j]
        R.append(acc / Wd[0][:, None])
    return R[r]
