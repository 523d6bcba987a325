"""Overlapping additive-Schwarz MFA encoder, literal per-subdomain form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, and where the paper says so
---------------------------------------------
* Plan (Section 2.2, eq. vecp-layout, Fig. 2-D schematic): the control grid is
  split into axis-aligned blocks of owned control points Omega_i.  Each block's
  free set F_i adds `overlap` control points on every interior side (the
  shared spans Delta plus the augmented spans delta; overlap >= max(1, floor(p/2))
  because Delta needs floor(p/2) spans for partition of unity).  The ghosts
  G_i are the p control points beyond F_i that the local data still touch;
  they carry the lagged neighbour values.  The local data D_i are all points
  in the support of some basis function in F_i, so each local normal-equation
  row equals the single-domain row.
* Sweep (Algorithm 1 "Domain Decomposed MFA Solver"; eq. global-system with
  the coupling blocks lambda at lagged iterates, which the text reads as a
  block-Jacobi / restricted additive Schwarz step): for every subdomain,
  independently, decode the current spline on D_i, form the residual against
  Q, and solve the unconstrained local least-squares problem
  (eq. minimization-problem) for a correction on F_i with the ghosts frozen.
  Starting from P = 0 the first sweep is the decoupled local fit of the
  algorithm's "if P_i = 0" branch.
* Combine (Section 2.3.2, uniform weights w = 1/n_s): every control point takes
  the average of the local solutions of all n_s subdomains whose F contains
  it, face and diagonal (multi-shared) neighbours alike.  A restricted variant
  (owner only) is also provided.
* Jump metric (eq. nonlinear-residuals, the interface terms F_ij): at the
  interface between neighbours i and j along axis a, the difference of the
  r-th derivatives (r = 0..p-1) along a of the two local solutions, evaluated
  on the data lines of i's owned range on the other axes.
* Fixed point: the converged multi-subdomain fit is the single-subdomain fit
  (Section 2.3, "same error profile as a single subdomain"); `global_direct`
  computes that fit directly.
* Weights (eq. nurbs-basis, W != 1; the conclusions' NURBS extension): with
  tensor-product weights W = w_0 x w_1 x w_2 the rational basis is the
  product of the per-axis rational bases, so every step above runs unchanged
  on the rational collocation matrices.  The weights are global, so averaging
  P or P W over the subdomains is the same combine.

Readings where the paper is silent are listed in the design notes of the
repository; the important ones are restated next to the code below.
"""
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List

import numpy as np

from . import bspline, lsq


# ----------------------------------------------------------------------------
# plan
# ----------------------------------------------------------------------------
@dataclass
class Block:
    c0: int          # owned control points [c0, c1)
    c1: int
    F0: int          # free set F = [F0, F1)
    F1: int
    E0: int          # F plus ghosts G: [E0, E1)
    E1: int
    D0: int          # local data points [D0, D1)
    D1: int
    own0: int        # owned data points [own0, own1) (a partition of the axis)
    own1: int


@dataclass
class AxisPlan:
    m: int
    n: int
    p: int
    overlap: int
    knots: np.ndarray
    u: np.ndarray
    span: np.ndarray
    blocks: List[Block]
    ns: np.ndarray                    # n_s per control point along this axis
    ustar: List[Fraction] = field(default_factory=list)   # interface params
    weights: np.ndarray = None        # NURBS weights of the axis (None: all 1)

    def coll(self, u, r=0):
        """Collocation (r-th derivative) of this axis' basis at parameters u."""
        return bspline.rational_collocation(self.knots, self.n, self.p, u, self.weights, r)


def min_overlap(p):
    """Smallest admissible overlap: the floor(p/2) shared spans of Delta, at least 1."""
    return max(1, p // 2)


def plan_axis(m, p, sizes, overlap, weights=None):
    """Plan one axis: m data points, owned control counts `sizes` per block,
    optional NURBS weights (one positive value per control point)."""
    sizes = [int(s) for s in sizes]
    n = sum(sizes)
    nb = len(sizes)
    if p < 1:
        raise ValueError("degree must be >= 1")
    if nb > 1 and overlap < min_overlap(p):
        raise ValueError("overlap below max(1, floor(p/2))")
    if overlap < 0:
        raise ValueError("negative overlap")
    if nb > 1 and min(sizes) < max(p + 1, 2 * overlap):
        raise ValueError("owned block smaller than max(p+1, 2*overlap)")
    if n < p + 1:
        raise ValueError("fewer than p+1 control points")
    if m < n:
        raise ValueError("fewer data points than control points")
    t = bspline.clamped_uniform_knots(n, p)
    u = bspline.params(m)
    span = bspline.find_span(t, n, p, u)

    # interfaces: Greville midpoint between the last owned control point of
    # block b and the first of block b+1, as exact rationals
    ustar = []
    c = 0
    for b in range(nb - 1):
        c += sizes[b]
        ustar.append((bspline.greville_fraction(n, p, c - 1)
                      + bspline.greville_fraction(n, p, c)) / 2)

    def first_point_at_or_after(fr):
        # smallest i with i/(m-1) >= fr
        i = 0
        while i < m and Fraction(i, m - 1) < fr:
            i += 1
        return i

    cuts = [0] + [first_point_at_or_after(us) for us in ustar] + [m]

    blocks = []
    c0 = 0
    for b in range(nb):
        c1 = c0 + sizes[b]
        F0 = max(0, c0 - overlap) if b > 0 else 0
        F1 = min(n, c1 + overlap) if b < nb - 1 else n
        E0 = max(0, F0 - p)
        E1 = min(n, F1 + p)
        smin = max(p, F0)
        smax = min(n - 1, F1 - 1 + p)
        idx = np.nonzero((span >= smin) & (span <= smax))[0]
        blocks.append(Block(c0, c1, F0, F1, E0, E1, int(idx[0]), int(idx[-1]) + 1,
                            cuts[b], cuts[b + 1]))
        c0 = c1
    ns = np.zeros(n, dtype=np.int64)
    for bl in blocks:
        ns[bl.F0:bl.F1] += 1
    if weights is not None:
        weights = np.asarray(weights, dtype=np.float64)
        if weights.shape != (n,) or not np.all(np.isfinite(weights)) or not np.all(weights > 0):
            raise ValueError("weights must be n positive finite values")
    return AxisPlan(m, n, p, overlap, t, u, span, blocks, ns, ustar, weights)


@dataclass
class Plan:
    axes: List[AxisPlan]
    p: int
    combine: str = "avg"

    @property
    def dim(self):
        return len(self.axes)

    @property
    def nsub(self):
        return tuple(len(a.blocks) for a in self.axes)

    @property
    def nctrl(self):
        return tuple(a.n for a in self.axes)


def make_plan(npts, p, sizes_per_axis, overlap, combine="avg", weights=None):
    """Plan a d-D problem: npts[a] points and owned sizes per block on axis a;
    weights: None, or per axis None or n_a positive NURBS weights."""
    if combine not in ("avg", "ras"):
        raise ValueError("combine must be 'avg' or 'ras'")
    ws = weights if weights is not None else [None] * len(npts)
    axes = [plan_axis(m, p, s, overlap, wa) for m, s, wa in zip(npts, sizes_per_axis, ws)]
    return Plan(axes, p, combine)


# ----------------------------------------------------------------------------
# setup: collocation matrices and local factors ("compute R" in Algorithm 1)
# ----------------------------------------------------------------------------
@dataclass
class Setup:
    plan: Plan
    colls: list          # per axis dense collocation matrix (m, n)
    factors: dict        # (axis, block) -> banded Cholesky factor of the local Gram


def setup(plan):
    colls = [ax.coll(ax.u) for ax in plan.axes]
    factors = {}
    for a, ax in enumerate(plan.axes):
        for b, bl in enumerate(ax.blocks):
            NF = colls[a][bl.D0:bl.D1, bl.F0:bl.F1]
            factors[(a, b)] = lsq.cholesky_band(lsq.gram_band(NF, plan.p))
    return Setup(plan, colls, factors)


# ----------------------------------------------------------------------------
# one Schwarz sweep
# ----------------------------------------------------------------------------
def local_corrections(S, Q, P):
    """Per-subdomain corrections dP_i on F_i (the local LSQ solves of one sweep).

    For subdomain i: r_i = Q[D_i] - N[D_i, E_i] P[E_i] (ghost values lagged),
    then dP_i = argmin ||r_i - N[D_i, F_i] x||, solved through the local normal
    equations with the banded Cholesky factor of each axis.
    Returns (dict idx -> dP_i, max |N[D_i,F_i]^T r_i| over all i).
    """
    plan = S.plan
    out = {}
    nres = 0.0
    for idx in np.ndindex(*plan.nsub):
        blks = [plan.axes[a].blocks[idx[a]] for a in range(plan.dim)]
        Dsl = tuple(slice(b.D0, b.D1) for b in blks)
        Esl = tuple(slice(b.E0, b.E1) for b in blks)
        NE = [S.colls[a][b.D0:b.D1, b.E0:b.E1] for a, b in enumerate(blks)]
        NF = [S.colls[a][b.D0:b.D1, b.F0:b.F1] for a, b in enumerate(blks)]
        r = Q[Dsl] - lsq.tensor_apply(NE, P[Esl])
        rhs = lsq.tensor_apply([N.T for N in NF], r)
        nres = max(nres, float(np.max(np.abs(rhs))))
        for a in range(plan.dim):
            rhs = lsq.solve_band_cholesky(S.factors[(a, idx[a])], rhs, axis=a)
        out[idx] = rhs
    return out, nres


def combine(S, P, dPs):
    """New consensus from the local solutions L_i = P + dP_i on F_i.

    'avg': P_new[k] = sum_{i: k in F_i} L_i[k] / n_s(k) (uniform weights);
    'ras': P_new[k] = L_owner(k)[k] (restricted to the owning subdomain).
    """
    plan = S.plan
    acc = np.zeros_like(P)
    cnt = np.zeros_like(P)
    for idx, dP in dPs.items():
        blks = [plan.axes[a].blocks[idx[a]] for a in range(plan.dim)]
        if plan.combine == "avg":
            sl = tuple(slice(b.F0, b.F1) for b in blks)
            acc[sl] += P[sl] + dP
            cnt[sl] += 1.0
        else:
            sl = tuple(slice(b.c0, b.c1) for b in blks)
            off = tuple(slice(b.c0 - b.F0, b.c1 - b.F0) for b in blks)
            acc[sl] += P[sl] + dP[off]
            cnt[sl] += 1.0
    assert np.all(cnt > 0)
    return acc / cnt


def jump_metric(S, dPs, P_new):
    """Normalised interface jumps J_r, r = 0..p-1 (max over axes and interfaces).

    Between neighbours i (block b) and j (block b+1) along axis a the two local
    solutions differ by ext(dP_i) - ext(dP_j) (both share the lagged P).  The
    r-th derivative along a of that difference is evaluated at the interface
    parameter u*_b and on the data points of i's owned range on every other
    axis; J_r^a is the largest magnitude found.  Each J_r^a is divided by
    max(S_r^a, S_0), where S_r^a is the largest r-th derivative control
    coefficient of the new consensus along a (a bound on max |d^r f/du_a^r|)
    and S_0 = max |P|.
    Returns (normalised J per r, raw J per axis and r).
    """
    plan = S.plan
    p = plan.p
    raw = np.zeros((plan.dim, p))
    for a, ax in enumerate(plan.axes):
        for b in range(len(ax.blocks) - 1):
            bi, bj = ax.blocks[b], ax.blocks[b + 1]
            lo, hi = bi.F0, bj.F1
            us = np.array([float(ax.ustar[b])])
            drows = [ax.coll(us, r)[0, lo:hi] for r in range(p)]
            for idx in np.ndindex(*plan.nsub):
                if idx[a] != b:
                    continue
                jdx = idx[:a] + (b + 1,) + idx[a + 1:]
                di = np.moveaxis(dPs[idx], a, 0)
                dj = np.moveaxis(dPs[jdx], a, 0)
                diff = np.zeros((hi - lo,) + di.shape[1:])
                diff[bi.F0 - lo:bi.F1 - lo] += di
                diff[bj.F0 - lo:bj.F1 - lo] -= dj
                others = [c for c in range(plan.dim) if c != a]
                for r in range(p):
                    T = np.tensordot(drows[r], diff, axes=([0], [0]))
                    for k, c in enumerate(others):
                        blc = plan.axes[c].blocks[idx[c]]
                        Nown = S.colls[c][blc.own0:blc.own1, blc.F0:blc.F1]
                        T = lsq.mode_product(Nown, T, k)
                    raw[a, r] = max(raw[a, r], float(np.max(np.abs(T))) if T.size else 0.0)
    S0 = float(np.max(np.abs(P_new)))
    norm = np.zeros(p)
    for a, ax in enumerate(plan.axes):
        for r in range(p):
            Sr = float(np.max(np.abs(bspline.derivative_coefficients(
                P_new, ax.knots, p, r, axis=a))))
            den = max(Sr, S0)
            val = raw[a, r] / den if den > 0 else 0.0
            norm[r] = max(norm[r], val)
    return norm, raw


@dataclass
class SweepStats:
    sweep: int
    jump: np.ndarray      # normalised J_r, r = 0..p-1
    max_dP: float         # max |P_new - P|
    nres_max: float       # max |N_F^T r| over subdomains, before the update


def sweep(S, Q, P, k=1):
    """One additive-Schwarz sweep: local corrections, combine, jump metric."""
    dPs, nres = local_corrections(S, Q, P)
    P_new = combine(S, P, dPs)
    jn, _ = jump_metric(S, dPs, P_new)
    return P_new, SweepStats(k, jn, float(np.max(np.abs(P_new - P))), nres)


def encode(S, Q, max_sweeps, jump_tol=None, P0=None):
    """Algorithm 1: sweep from P0 (default 0) until max_r J_r < jump_tol or max_sweeps."""
    Q = np.asarray(Q, dtype=np.float64)
    P = np.zeros(S.plan.nctrl) if P0 is None else np.array(P0, dtype=np.float64)
    hist = []
    for k in range(1, max_sweeps + 1):
        P, st = sweep(S, Q, P, k)
        hist.append(st)
        if jump_tol is not None and float(np.max(st.jump)) < jump_tol:
            break
    return P, hist


def decode(S, P, derivs=None):
    """Evaluate the spline (or a mixed partial derivative) on the full grid."""
    plan = S.plan
    mats = []
    for a, ax in enumerate(plan.axes):
        r = 0 if derivs is None else derivs[a]
        mats.append(S.colls[a] if r == 0 else ax.coll(ax.u, r))
    return lsq.tensor_apply(mats, P)


def global_direct(S, Q):
    """Single-domain least-squares fit: the fixed point of the iteration."""
    return lsq.separable_lsq(np.asarray(Q, dtype=np.float64), S.colls, S.plan.p)
