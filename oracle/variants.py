"""The two alternatives to floating interface knots that the paper compares
against (Section 2.1; Section 3.1.1 "Comparison of Clamped vs Floating
Boundary Knots"; the error-profile figure at the interface).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Decoupled local fits
--------------------
Every subdomain solves its unconstrained least-squares problem (eq.
minimization-problem) on its own data, without any exchange: Algorithm 1's
branch for P_i = 0 before the constraint iterations.  With the floating knots
of Section 2.2 this is the local fit over the free set F_i with the data D_i
in its support (ghosts zero).  The result is one spline per subdomain; the
decoded field takes, at each data point, the spline of the subdomain that
owns the point, so it is discontinuous at the interfaces.

Clamped interfaces (C^0)
------------------------
Every subdomain has its own clamped knot vector (p+1 repeated knots at both
of its ends, uniform inside) and its own control points; neighbours share the
control point that sits on their common interface, and that control point
interpolates the input datum there (Section 2.1: the common control points at
subdomain interfaces are clamped to input data points).  The decoded field is
therefore C^0 but in general not C^1 across an interface.  Readings taken:
  * a block's local parameter is v = (i - a0) / (a1 - a0) for data index i
    between its interface indices a0 < a1, so d/du = (m - 1) / (a1 - a0) d/dv;
  * the interfaces of an axis sit on data points: with n_b control points and
    n_b - p spans in block b, interface b lies at the data index closest to
    (m - 1) * (spans of blocks before b) / (all spans), halves rounded up;
    block b covers the data points between its two interfaces, both
    included, and owns those from its left interface up to (not including)
    its right one (the last block owns its right end too);
  * in d dimensions the shared lower-dimensional entities are fitted first
    and then frozen: vertices take the data value, every interface edge is a
    1-D least-squares fit of the data on it with its end vertices fixed,
    every interface face a 2-D fit with its edges fixed, and every subdomain
    interior a d-D fit with its whole boundary frame fixed.  Here each of
    these fits is a dense least-squares solve on the Kronecker product of the
    collocation matrices, with the frozen control points moved to the right
    hand side (slow and literal).
"""
from dataclasses import dataclass
from itertools import product
from typing import List

import numpy as np

from . import bspline, lsq, schwarz


# ----------------------------------------------------------------------------
# decoupled local fits (floating knots, no exchange)
# ----------------------------------------------------------------------------
def decoupled_fit(S, Q):
    """Local least-squares fit of every subdomain over its free set F_i and
    its data D_i, ghosts zero: {idx: control points on F_i}."""
    P0 = np.zeros(S.plan.nctrl)
    fits, _ = schwarz.local_corrections(S, np.asarray(Q, dtype=np.float64), P0)
    return fits


def decoupled_decode(S, fits, derivs=None):
    """Decode of the decoupled model: every data point takes the spline of
    the subdomain that owns it (owned ranges partition each axis)."""
    plan = S.plan
    out = np.zeros(tuple(ax.m for ax in plan.axes))
    for idx, L in fits.items():
        blks = [plan.axes[a].blocks[idx[a]] for a in range(plan.dim)]
        mats = []
        for a, (ax, bl) in enumerate(zip(plan.axes, blks)):
            r = 0 if derivs is None else derivs[a]
            C = S.colls[a] if r == 0 else ax.coll(ax.u, r)
            mats.append(C[bl.own0:bl.own1, bl.F0:bl.F1])
        out[tuple(slice(bl.own0, bl.own1) for bl in blks)] = lsq.tensor_apply(mats, L)
    return out


def decoupled_jumps(S, fits):
    """Raw interface jumps of the decoupled model: for neighbours i, j along
    axis a, max |d^r/du_a^r (f_i - f_j)| at the interface parameter u* over
    the data points of i's owned range on the other axes, r = 0..p-1.
    Returns an array (dim, p)."""
    plan = S.plan
    p = plan.p
    raw = np.zeros((plan.dim, p))
    for a, ax in enumerate(plan.axes):
        for b in range(len(ax.blocks) - 1):
            bi, bj = ax.blocks[b], ax.blocks[b + 1]
            us = np.array([float(ax.ustar[b])])
            for idx in np.ndindex(*plan.nsub):
                if idx[a] != b:
                    continue
                jdx = idx[:a] + (b + 1,) + idx[a + 1:]
                for r in range(p):
                    row = ax.coll(us, r)[0]
                    vi = np.tensordot(row[bi.F0:bi.F1], fits[idx], axes=([0], [a]))
                    vj = np.tensordot(row[bj.F0:bj.F1], fits[jdx], axes=([0], [a]))
                    T = vi - vj
                    others = [c for c in range(plan.dim) if c != a]
                    for k, c in enumerate(others):
                        blc = plan.axes[c].blocks[idx[c]]
                        T = lsq.mode_product(S.colls[c][blc.own0:blc.own1, blc.F0:blc.F1], T, k)
                    raw[a, r] = max(raw[a, r], float(np.max(np.abs(T))) if T.size else 0.0)
    return raw


# ----------------------------------------------------------------------------
# clamped interfaces (C^0)
# ----------------------------------------------------------------------------
@dataclass
class ClampedAxis:
    m: int
    p: int
    sizes: List[int]      # control points of each block (shared ends counted in both)
    cuts: List[int]       # data index of each block boundary (cuts[0] = 0, cuts[B] = m - 1)
    offs: List[int]       # global index of each block's first control point
    n: int                # control points of the axis: sum(sizes) - (B - 1)

    @property
    def nblocks(self):
        return len(self.sizes)

    def owned(self, b):
        """Data points owned by block b: [cuts[b], cuts[b+1]) (the last block
        includes m - 1)."""
        return self.cuts[b], (self.cuts[b + 1] if b < self.nblocks - 1 else self.m)

    def local_rows(self, b, i0, i1, r=0):
        """Rows of block b's basis (its own clamped knots, derivative r with
        respect to the global parameter u) at data points i0..i1-1."""
        nb = self.sizes[b]
        t = bspline.clamped_uniform_knots(nb, self.p)
        a0, a1 = self.cuts[b], self.cuts[b + 1]
        # local parameter from the integer indices, so that a point on a
        # local knot lands exactly on it: v = (i - a0) / (a1 - a0)
        v = np.clip((np.arange(i0, i1) - a0) / (a1 - a0), 0.0, 1.0)
        return bspline.collocation(t, nb, self.p, v, r) * ((self.m - 1) / (a1 - a0)) ** r

    def collocation(self, r=0):
        """Piecewise collocation (m, n): each data point uses its owner block."""
        C = np.zeros((self.m, self.n))
        for b in range(self.nblocks):
            i0, i1 = self.owned(b)
            C[i0:i1, self.offs[b]:self.offs[b] + self.sizes[b]] = self.local_rows(b, i0, i1, r)
        return C


def plan_clamped_axis(m, p, sizes):
    """Blocks of `sizes` control points with their own clamped knots; the
    interfaces sit on data points in proportion to the blocks' span counts."""
    sizes = [int(s) for s in sizes]
    B = len(sizes)
    if min(sizes) < p + 1:
        raise ValueError("a block needs at least p+1 control points")
    spans = [s - p for s in sizes]
    tot = sum(spans)
    cuts = [0]
    acc = 0
    for b in range(B - 1):
        acc += spans[b]
        cuts.append(((m - 1) * acc * 2 + tot) // (2 * tot))
    cuts.append(m - 1)
    for b in range(B):
        if cuts[b + 1] - cuts[b] + 1 < sizes[b]:
            raise ValueError("a block has fewer data points than control points")
    offs = [0]
    for b in range(B - 1):
        offs.append(offs[-1] + sizes[b] - 1)
    return ClampedAxis(m, p, sizes, cuts, offs, sum(sizes) - (B - 1))


def plan_clamped(npts, p, sizes_per_axis):
    return [plan_clamped_axis(m, p, s) for m, s in zip(npts, sizes_per_axis)]


def _parts(ax):
    """The pieces of one axis: ('I', b) the interface after block b (one
    shared control point, one data point), ('F', b) block b without its
    interface ends."""
    out = [("F", b) for b in range(ax.nblocks)]
    out += [("I", b) for b in range(ax.nblocks - 1)]
    return out


def _part_data_ctrl(ax, part):
    """(data indices, all control points of the part's closure, the part's
    own unknown control points) as global indices."""
    kind, b = part
    if kind == "I":
        g = ax.offs[b + 1]
        return np.array([ax.cuts[b + 1]]), np.array([g]), np.array([g])
    i0, i1 = ax.cuts[b], ax.cuts[b + 1] + 1
    closure = np.arange(ax.offs[b], ax.offs[b] + ax.sizes[b])
    lo = 1 if b > 0 else 0
    hi = ax.sizes[b] - 1 if b < ax.nblocks - 1 else ax.sizes[b]
    return np.arange(i0, i1), closure, closure[lo:hi]


def _part_rows(ax, part):
    """Collocation of the part's closure at its data points."""
    kind, b = part
    if kind == "I":
        return np.ones((1, 1))
    return ax.local_rows(b, ax.cuts[b], ax.cuts[b + 1] + 1)


def clamped_fit(axes, Q):
    """Control points (n_0 x ... ) of the clamped-interface fit, entity by
    entity in order of decreasing number of interface axes."""
    Q = np.asarray(Q, dtype=np.float64)
    dim = len(axes)
    P = np.zeros(tuple(ax.n for ax in axes))
    done = np.zeros(P.shape, dtype=bool)
    ents = list(product(*[_parts(ax) for ax in axes]))
    ents.sort(key=lambda e: -sum(1 for k, _ in e if k == "I"))
    for ent in ents:
        info = [_part_data_ctrl(ax, pt) for ax, pt in zip(axes, ent)]
        rows = [_part_rows(ax, pt) for ax, pt in zip(axes, ent)]
        data = Q[np.ix_(*[d for d, _, _ in info])].ravel()
        K = rows[0]
        for R in rows[1:]:
            K = np.kron(K, R)
        # columns of K enumerate the closure in C order
        grids = np.meshgrid(*[c for _, c, _ in info], indexing="ij")
        cols = [g.ravel() for g in grids]
        unknown = np.ones(len(cols[0]), dtype=bool)
        for a, (_, c, u) in enumerate(info):
            unknown &= np.isin(cols[a], u)
        known_idx = tuple(cl[~unknown] for cl in cols)
        assert np.all(done[known_idx]), "frame not fitted before the entity"
        rhs = data - K[:, ~unknown] @ P[known_idx]
        x = np.linalg.lstsq(K[:, unknown], rhs, rcond=None)[0]
        uidx = tuple(cl[unknown] for cl in cols)
        P[uidx] = x
        done[uidx] = True
    assert np.all(done)
    return P


def clamped_decode(axes, P, derivs=None):
    mats = [ax.collocation(0 if derivs is None else derivs[a]) for a, ax in enumerate(axes)]
    return lsq.tensor_apply(mats, P)


def clamped_jumps(axes, P):
    """Raw interface jumps of the clamped model: at the interface after
    block b along axis a, max |d^r/du_a^r (f_b - f_{b+1})| (block b's end
    against block b+1's start) over the data points of the other axes,
    r = 0..p-1.  Returns an array (dim, p)."""
    dim = len(axes)
    p = axes[0].p
    raw = np.zeros((dim, p))
    for a, ax in enumerate(axes):
        for b in range(ax.nblocks - 1):
            i = ax.cuts[b + 1]
            for r in range(p):
                row = np.zeros(ax.n)
                row[ax.offs[b]:ax.offs[b] + ax.sizes[b]] += ax.local_rows(b, i, i + 1, r)[0]
                row[ax.offs[b + 1]:ax.offs[b + 1] + ax.sizes[b + 1]] -= \
                    ax.local_rows(b + 1, i, i + 1, r)[0]
                T = np.tensordot(row, P, axes=([0], [a]))
                others = [c for c in range(dim) if c != a]
                for k, c in enumerate(others):
                    T = lsq.mode_product(axes[c].collocation(0), T, k)
                raw[a, r] = max(raw[a, r], float(np.max(np.abs(T))))
    return raw
