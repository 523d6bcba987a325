"""Pins of the oracle's decoupled and clamped-interface (C^0) variants.

Decoupled local fits: every subdomain's fit equals a brute-force dense
least-squares solve on the Kronecker product of its own collocation blocks;
one subdomain is the single-domain fit; the decoded field is discontinuous.

Clamped interfaces: the decoded field is continuous across every interface
(J_0 = 0) but its first derivative jumps; the shared control points take the
data at the interface vertices; polynomials of degree <= p are reproduced
exactly; one block per axis is the plain single-domain fit; in 1-D the fit
equals the constrained least-squares problem solved through its KKT system;
and the entity-by-entity fit equals the tensor product of one per-axis
operator (interface rows pick the datum, free rows are the block's
least-squares fit with its interface ends moved to the right-hand side).
"""
import numpy as np
import pytest

from oracle import bspline, lsq, schwarz, variants
from paper_2210_06528_amd import workloads as W


def _field(npts, seed=3):
    return W.field_spectral(npts, kmax=max(1, min(npts) // 6), seed=seed, dtype=np.float64)


# ------------------------------------------------------------------ decoupled
@pytest.mark.parametrize("npts,sizes", [((400,), [[12, 14, 13]]),
                                        ((61, 47), [[9, 9], [7, 8]])])
def test_decoupled_fits_equal_dense_lstsq(npts, sizes):
    plan = schwarz.make_plan(npts, 3, sizes, 2)
    S = schwarz.setup(plan)
    Q = _field(npts)
    fits = variants.decoupled_fit(S, Q)
    for idx, L in fits.items():
        blks = [plan.axes[a].blocks[idx[a]] for a in range(plan.dim)]
        mats = [S.colls[a][b.D0:b.D1, b.F0:b.F1] for a, b in enumerate(blks)]
        K = mats[0]
        for M in mats[1:]:
            K = np.kron(K, M)
        y = Q[tuple(slice(b.D0, b.D1) for b in blks)].ravel()
        ref = np.linalg.lstsq(K, y, rcond=None)[0].reshape(L.shape)
        assert np.max(np.abs(L - ref)) < 1e-10 * np.max(np.abs(ref))


def test_decoupled_one_subdomain_is_the_single_fit_and_blocks_are_discontinuous():
    npts = (300,)
    Q = _field(npts)
    S1 = schwarz.setup(schwarz.make_plan(npts, 3, [[40]], 2))
    f1 = variants.decoupled_decode(S1, variants.decoupled_fit(S1, Q))
    ref = schwarz.decode(S1, schwarz.global_direct(S1, Q))
    assert np.max(np.abs(f1 - ref)) < 1e-12
    S = schwarz.setup(schwarz.make_plan(npts, 3, [[20, 20]], 2))
    raw = variants.decoupled_jumps(S, variants.decoupled_fit(S, Q))
    assert raw[0, 0] > 1e-6


# ------------------------------------------------------------------ clamped
@pytest.mark.parametrize("npts,sizes", [((401,), [[12, 14, 13]]),
                                        ((61, 47), [[9, 9], [7, 8, 7]]),
                                        ((30, 27, 25), [[7, 8], [7, 7], [6, 7]])])
def test_clamped_is_c0_not_c1_and_interpolates_interface_vertices(npts, sizes):
    axes = variants.plan_clamped(npts, 3, sizes)
    Q = _field(npts)
    P = variants.clamped_fit(axes, Q)
    raw = variants.clamped_jumps(axes, P)
    assert np.max(raw[:, 0]) < 1e-12 * np.max(np.abs(P))
    assert np.max(raw[:, 1]) > 1e-6
    # vertices: every axis at an interface -> the control point is the datum
    import itertools
    ifs = [[(ax.offs[b + 1], ax.cuts[b + 1]) for b in range(ax.nblocks - 1)] for ax in axes]
    for combo in itertools.product(*ifs):
        g = tuple(c[0] for c in combo)
        i = tuple(c[1] for c in combo)
        assert abs(P[g] - Q[i]) < 1e-13


@pytest.mark.parametrize("npts,sizes", [((200,), [[9, 11]]), ((45, 38), [[8, 9], [7, 8]])])
def test_clamped_reproduces_polynomials(npts, sizes):
    p = 3
    axes = variants.plan_clamped(npts, p, sizes)
    us = np.meshgrid(*[np.arange(m) / (m - 1) for m in npts], indexing="ij")
    Q = np.ones(npts)
    for k, u in enumerate(us):
        Q = Q * (1.0 + (k + 1) * u - 0.7 * u ** 2 + 0.3 * u ** 3)
    P = variants.clamped_fit(axes, Q)
    assert np.max(np.abs(variants.clamped_decode(axes, P) - Q)) < 1e-11


def test_clamped_one_block_is_the_single_domain_fit():
    npts = (50, 41)
    Q = _field(npts)
    axes = variants.plan_clamped(npts, 3, [[12], [10]])
    P = variants.clamped_fit(axes, Q)
    S = schwarz.setup(schwarz.make_plan(npts, 3, [[12], [10]], 2))
    assert np.max(np.abs(P - schwarz.global_direct(S, Q))) < 1e-10 * np.max(np.abs(P))


def test_clamped_1d_equals_kkt_constrained_lstsq():
    m, p = 333, 3
    axes = variants.plan_clamped((m,), p, [[11, 13, 12]])
    ax = axes[0]
    Q = _field((m,), seed=9)
    N = ax.collocation()
    # constraints: the shared control points equal the data at the interfaces
    C = np.zeros((ax.nblocks - 1, ax.n))
    g = np.zeros(ax.nblocks - 1)
    for b in range(ax.nblocks - 1):
        C[b, ax.offs[b + 1]] = 1.0
        g[b] = Q[ax.cuts[b + 1]]
    KKT = np.block([[N.T @ N, C.T], [C, np.zeros((len(g), len(g)))]])
    sol = np.linalg.solve(KKT, np.concatenate([N.T @ Q, g]))
    P = variants.clamped_fit(axes, Q)
    assert np.max(np.abs(P - sol[:ax.n])) < 1e-10 * np.max(np.abs(P))


def _axis_operator(ax):
    """Per-axis clamped operator (n x m): interface rows pick the datum; the
    free rows of block b are its least-squares fit over its data with the
    interface ends' data moved to the right-hand side."""
    L = np.zeros((ax.n, ax.m))
    for b in range(ax.nblocks):
        i0, i1 = ax.cuts[b], ax.cuts[b + 1] + 1
        Nb = ax.local_rows(b, i0, i1)
        lo = 1 if b > 0 else 0
        hi = ax.sizes[b] - 1 if b < ax.nblocks - 1 else ax.sizes[b]
        Nf = Nb[:, lo:hi]
        Z = np.linalg.inv(Nf.T @ Nf) @ Nf.T          # (free, data)
        rows = Z.copy()
        if lo == 1:
            rows[:, 0] -= Z @ Nb[:, 0]
        if hi == ax.sizes[b] - 1:
            rows[:, -1] -= Z @ Nb[:, -1]
        L[ax.offs[b] + lo:ax.offs[b] + hi, i0:i1] = rows
        if b < ax.nblocks - 1:
            L[ax.offs[b + 1], ax.cuts[b + 1]] = 1.0
    return L


@pytest.mark.parametrize("npts,sizes", [((61, 47), [[9, 9], [7, 8, 7]]),
                                        ((30, 27, 25), [[7, 8], [7, 7], [6, 7]])])
def test_clamped_fit_is_separable(npts, sizes):
    axes = variants.plan_clamped(npts, 3, sizes)
    Q = _field(npts)
    P = variants.clamped_fit(axes, Q)
    Ps = lsq.tensor_apply([_axis_operator(ax) for ax in axes], Q)
    assert np.max(np.abs(P - Ps)) < 1e-10 * np.max(np.abs(P))


def test_clamped_plan_rejects_too_few_points():
    with pytest.raises(ValueError):
        variants.plan_clamped_axis(20, 3, [12, 12])
    with pytest.raises(ValueError):
        variants.plan_clamped_axis(200, 3, [3, 12])
