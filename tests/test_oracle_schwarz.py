"""Pins for the oracle's Schwarz iteration, combine, jump metric and fixed point.

Section 2.2 (plan, shared spans), eq. global-system and Section 2.3.2 (lagged
coupling = block Jacobi / additive Schwarz, uniform 1/n_s weights), Algorithm 1,
eq. nonlinear-residuals (interface jumps), and the single-subdomain fixed point
the paper uses as its accuracy reference.

The independent references are: dense matrices built from SciPy's design
matrix (the affine map of one weighted additive-Schwarz step on the global
normal equations), exact polynomial reproduction, mirror symmetry, and SciPy
derivatives for the jump metric.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline, lsq, schwarz
from paper_2210_06528_amd import workloads as W


def _design(n, p, m):
    t = bspline.clamped_uniform_knots(n, p)
    u = np.arange(m) / (m - 1)
    return BSpline.design_matrix(u, t, p).toarray()


def _free_ranges(sizes, o):
    out, c0 = [], 0
    for b, s in enumerate(sizes):
        c1 = c0 + s
        out.append((max(0, c0 - o) if b else 0, min(sum(sizes), c1 + o) if b < len(sizes) - 1
                    else sum(sizes), c0, c1))
        c0 = c1
    return out


def _dense_step_matrices(npts, p, sizes, o, combine):
    """A = kron C_a^T C_a and the weighted additive-Schwarz operator B, densely."""
    Cs = [_design(sum(s), p, m) for s, m in zip(sizes, npts)]
    C = Cs[0]
    for c in Cs[1:]:
        C = np.kron(C, c)
    A = C.T @ C
    nctrl = [sum(s) for s in sizes]
    N = int(np.prod(nctrl))
    ids = np.arange(N).reshape(nctrl)
    frs = [_free_ranges(s, o) for s in sizes]
    boxes = []
    for idx in np.ndindex(*[len(s) for s in sizes]):
        Fsl = tuple(slice(frs[a][b][0], frs[a][b][1]) for a, b in enumerate(idx))
        Osl = tuple(slice(frs[a][b][2], frs[a][b][3]) for a, b in enumerate(idx))
        boxes.append((ids[Fsl].ravel(), set(ids[Osl].ravel().tolist())))
    ns = np.zeros(N)
    for F, _ in boxes:
        ns[F] += 1
    B = np.zeros((N, N))
    for F, own in boxes:
        inv = np.linalg.inv(A[np.ix_(F, F)])
        if combine == "avg":
            w = 1.0 / ns[F]
        else:
            w = np.array([1.0 if k in own else 0.0 for k in F])
        B[np.ix_(F, F)] += w[:, None] * inv
    return C, A, B


@pytest.mark.parametrize("combine", ["avg", "ras"])
@pytest.mark.parametrize("npts,p,sizes,o", [
    ((60,), 3, [[6, 7, 6]], 2),
    ((45,), 2, [[5, 6, 5, 6]], 1),
    ((31, 27), 3, [[5, 6], [4, 5]], 2),
    ((23, 19, 21), 2, [[4, 4], [4, 4], [5, 4]], 2),
])
def test_sweep_is_dense_weighted_additive_schwarz(npts, p, sizes, o, combine):
    C, A, B = _dense_step_matrices(npts, p, sizes, o, combine)
    rng = np.random.default_rng(11)
    Q = rng.standard_normal(npts)
    P0 = rng.standard_normal([sum(s) for s in sizes])
    plan = schwarz.make_plan(npts, p, sizes, o, combine=combine)
    S = schwarz.setup(plan)
    P1, st = schwarz.sweep(S, Q, P0)
    g = C.T @ Q.ravel() - A @ P0.ravel()
    ref = P0.ravel() + B @ g
    assert np.max(np.abs(P1.ravel() - ref)) < 1e-10 * np.max(np.abs(ref))
    assert abs(st.nres_max - np.max(np.abs(g))) < 1e-10 * np.max(np.abs(g))


def test_contraction_equals_spectral_radius_1d():
    w = W.cfg_1d()
    C, A, B = _dense_step_matrices(w.npts, w.degree, w.sizes, w.overlap, "avg")
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - B @ A)))
    plan = schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap)
    S = schwarz.setup(plan)
    Q = W.make_field(w)
    Pstar = schwarz.global_direct(S, Q)
    P = np.zeros(80)
    errs = []
    for k in range(6):
        P, _ = schwarz.sweep(S, Q, P, k + 1)
        errs.append(np.linalg.norm(P - Pstar))
    ratios = [errs[k + 1] / errs[k] for k in range(2, 5)]
    assert abs(rho - 0.0154) < 5e-4
    assert all(abs(r - rho) < 0.1 * rho for r in ratios)


def test_cfg1_mirror_symmetry_every_sweep():
    w = W.cfg_1d()
    S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
    Q = W.make_field(w)
    assert np.max(np.abs(Q - Q[::-1])) < 1e-15
    Q = 0.5 * (Q + Q[::-1])            # exactly even input
    P = np.zeros(80)
    for k in range(10):
        P, st = schwarz.sweep(S, Q, P, k + 1)
        assert np.max(np.abs(P - P[::-1])) < 1e-13 * np.max(np.abs(P))


def test_cfg1_converges_to_direct():
    w = W.cfg_1d()
    S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
    Q = W.make_field(w)
    P, hist = schwarz.encode(S, Q, 10)
    Pstar = schwarz.global_direct(S, Q)
    assert len(hist) == 10
    assert np.max(np.abs(P - Pstar)) < 1e-13 * np.max(np.abs(Pstar))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_polynomial_reproduction(p):
    """Degree <= p per axis: the direct fit is exact, the exact fit is a fixed
    point of one sweep (zero jumps), and the iteration from P = 0 reaches it."""
    npts, sizes, o = (37, 29), [[6, 7, 6], [6, 6]], max(1, p // 2)
    sizes = [[max(s, p + 1, 2 * o) for s in ax] for ax in sizes]
    plan = schwarz.make_plan(npts, p, sizes, o)
    S = schwarz.setup(plan)
    u = [np.arange(m) / (m - 1) for m in npts]
    U, V = np.meshgrid(*u, indexing="ij")
    Q = 1.5 - U ** p + 2.0 * U * V ** max(0, p - 1) + V ** p * U
    Pstar = schwarz.global_direct(S, Q)
    assert np.max(np.abs(schwarz.decode(S, Pstar) - Q)) < 1e-12
    P1, st = schwarz.sweep(S, Q, Pstar)
    assert np.max(np.abs(P1 - Pstar)) < 1e-12
    assert np.max(st.jump) < 1e-10 and st.nres_max < 1e-11
    P, hist = schwarz.encode(S, Q, 200, jump_tol=1e-13)
    assert np.max(np.abs(schwarz.decode(S, P) - Q)) < 1e-11


def test_constant_and_linear_give_one_and_greville():
    p = 3
    plan = schwarz.make_plan((50,), p, [[6, 7, 6]], 2)
    S = schwarz.setup(plan)
    P, _ = schwarz.encode(S, np.ones(50), 60, jump_tol=1e-14)
    assert np.max(np.abs(P - 1.0)) < 1e-13
    u = np.arange(50) / 49
    P, _ = schwarz.encode(S, u, 60, jump_tol=1e-14)
    ax = plan.axes[0]
    assert np.max(np.abs(P - bspline.greville(ax.knots, ax.n, p))) < 1e-13


def test_single_subdomain_exact_in_one_sweep():
    w = W.small_3d(sizes=((14,), (12,), (11,)))
    plan = schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap)
    S = schwarz.setup(plan)
    Q = W.make_field(w)
    P, hist = schwarz.encode(S, Q, 1)
    assert np.max(np.abs(P - schwarz.global_direct(S, Q))) < 1e-12 * np.max(np.abs(P))


@pytest.mark.parametrize("combine", ["avg", "ras"])
def test_fixed_point_is_single_domain_fit(combine):
    w = W.small_3d()
    plan = schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap, combine=combine)
    S = schwarz.setup(plan)
    Q = W.make_field(w)
    P, hist = schwarz.encode(S, Q, 80, jump_tol=1e-12)
    Pstar = schwarz.global_direct(S, Q)
    assert np.max(hist[-1].jump) < 1e-12
    assert np.max(np.abs(P - Pstar)) < 1e-10 * np.max(np.abs(Pstar))


def test_jump_metric_matches_scipy_derivatives_2d():
    npts, p, sizes, o = (41, 33), 3, [[7, 8], [6, 6]], 2
    plan = schwarz.make_plan(npts, p, sizes, o)
    S = schwarz.setup(plan)
    rng = np.random.default_rng(4)
    dPs = {}
    for idx in np.ndindex(*plan.nsub):
        shp = tuple(plan.axes[a].blocks[idx[a]].F1 - plan.axes[a].blocks[idx[a]].F0
                    for a in range(2))
        dPs[idx] = rng.standard_normal(shp)
    P = rng.standard_normal(plan.nctrl)
    _, raw = schwarz.jump_metric(S, dPs, P)
    # axis-0 interface between blocks (0, by) and (1, by), recomputed with SciPy
    ax0, ax1 = plan.axes
    want = np.zeros(p)
    us = float(ax0.ustar[0])
    for by in range(2):
        bi, bj = ax0.blocks[0], ax0.blocks[1]
        byb = ax1.blocks[by]
        diff = np.zeros((ax0.n, byb.F1 - byb.F0))
        diff[bi.F0:bi.F1] += dPs[(0, by)]
        diff[bj.F0:bj.F1] -= dPs[(1, by)]
        yrows = BSpline.design_matrix(ax1.u[byb.own0:byb.own1], ax1.knots, p).toarray()
        yrows = yrows[:, byb.F0:byb.F1]
        for r in range(p):
            vals = np.array([(BSpline(ax0.knots, diff[:, k], p).derivative(r)(us) if r else
                              BSpline(ax0.knots, diff[:, k], p)(us))
                             for k in range(diff.shape[1])])
            want[r] = max(want[r], np.max(np.abs(yrows @ vals)))
    assert np.allclose(raw[0], want, rtol=1e-10, atol=1e-12)


def test_interface_is_greville_midpoint_and_owned_ranges_partition():
    plan = schwarz.make_plan((2000,), 3, [[40, 40]], 3)
    ax = plan.axes[0]
    # symmetric split: interface at the centre of [0, 1]
    assert ax.ustar[0] == Fraction(1, 2)
    assert ax.blocks[0].own1 == 1000 and ax.blocks[1].own0 == 1000
    w = W.cfg_3d_mixed()
    plan = schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap)
    for ax in plan.axes:
        assert ax.blocks[0].own0 == 0 and ax.blocks[-1].own1 == ax.m
        for a, b in zip(ax.blocks, ax.blocks[1:]):
            assert a.own1 == b.own0
            assert a.D0 <= a.own0 and a.own1 <= a.D1


def test_plan_rejects_bad_input():
    with pytest.raises(ValueError):
        schwarz.make_plan((100,), 3, [[10, 10]], 0)        # overlap below minimum
    with pytest.raises(ValueError):
        schwarz.make_plan((100,), 4, [[10, 10]], 1)        # p=4 needs overlap >= 2
    with pytest.raises(ValueError):
        schwarz.make_plan((100,), 3, [[3, 17]], 1)         # block smaller than p+1
    with pytest.raises(ValueError):
        schwarz.make_plan((10,), 3, [[8, 8]], 1)           # fewer points than ctrl


@pytest.mark.parametrize("p", [2, 3, 4])
def test_more_overlap_contracts_faster(p):
    """Section 3.1.2 / Section 2.2: augmented overlap improves convergence."""
    npts, sizes = (240,), [[8, 8, 8]]
    rhos = []
    for o in (0, 1, 2, 3):
        C, A, B = _dense_step_matrices(npts, p, sizes, o, "avg")
        rhos.append(np.max(np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - B @ A))))
    assert all(r < 1.0 for r in rhos)
    assert all(a > b for a, b in zip(rhos, rhos[1:]))


# ----------------------------------------------------------------------------
# jump metric (eq. nonlinear-residuals) recomputed with SciPy, 3-D, all axes
# ----------------------------------------------------------------------------
_J3 = dict(npts=(26, 23, 21), p=3, sizes=[[5, 6, 5], [5, 6], [6, 5]], o=2)


def _embed(block_vals, blks, nctrl):
    """A block's F-range array placed into a zero control array of full size."""
    full = np.zeros(nctrl)
    full[tuple(slice(b.F0, b.F1) for b in blks)] = block_vals
    return full


def _scipy_raw_jumps(plan, dPs):
    """max |d^r/du_a^r (ext dP_i - ext dP_j)| at u*, over the data points of
    i's owned range on every other axis, evaluated with SciPy's BSpline
    (derivative of the spline along a, plain evaluation along the others)."""
    p, d = plan.p, plan.dim
    raw = np.zeros((d, p))
    for a, ax in enumerate(plan.axes):
        for b in range(len(ax.blocks) - 1):
            us = float(ax.ustar[b])
            for idx in np.ndindex(*plan.nsub):
                if idx[a] != b:
                    continue
                jdx = idx[:a] + (b + 1,) + idx[a + 1:]
                bi = [plan.axes[c].blocks[idx[c]] for c in range(d)]
                bj = [plan.axes[c].blocks[jdx[c]] for c in range(d)]
                diff = _embed(dPs[idx], bi, plan.nctrl) - _embed(dPs[jdx], bj, plan.nctrl)
                for r in range(p):
                    spl = BSpline(ax.knots, diff, p, axis=a)
                    vals = (spl.derivative(r) if r else spl)(us)   # axis a removed
                    for c in range(d):
                        if c == a:
                            continue
                        cc = c if c < a else c - 1                  # position in vals
                        axc = plan.axes[c]
                        own = axc.u[bi[c].own0:bi[c].own1]
                        vals = np.moveaxis(BSpline(axc.knots, vals, p, axis=cc)(own), 0, cc)
                    raw[a, r] = max(raw[a, r], float(np.max(np.abs(vals))))
    return raw


def _random_local(plan, rng, scale=1.0):
    dPs = {}
    for idx in np.ndindex(*plan.nsub):
        shp = tuple(plan.axes[a].blocks[idx[a]].F1 - plan.axes[a].blocks[idx[a]].F0
                    for a in range(plan.dim))
        dPs[idx] = scale * rng.standard_normal(shp)
    return dPs


def test_jump_metric_raw_matches_scipy_3d_all_axes():
    plan = schwarz.make_plan(_J3["npts"], _J3["p"], _J3["sizes"], _J3["o"])
    S = schwarz.setup(plan)
    rng = np.random.default_rng(21)
    dPs = _random_local(plan, rng)
    _, raw = schwarz.jump_metric(S, dPs, rng.standard_normal(plan.nctrl))
    want = _scipy_raw_jumps(plan, dPs)
    assert np.all(want > 0)
    assert np.allclose(raw, want, rtol=1e-10, atol=0), (raw, want)


def _anisotropic(plan, rng):
    """Control array whose derivative scales differ by axis: smooth along
    axis 0, rough along axis 1, a ramp along axis 2."""
    g = [np.linspace(0.0, 1.0, n) for n in plan.nctrl]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    return (np.sin(2.0 * X) + 0.3 * rng.standard_normal(plan.nctrl) * (1.0 + Y)
            + 5.0 * Z)


def test_sweep_jump_normalisation_uses_new_consensus_per_axis():
    """The normalised jump of a sweep is max_a raw_a,r / max(S_r^a, S_0), with
    S_r^a the largest r-th derivative control coefficient along axis a of the
    NEW consensus (SciPy's derivative spline) and S_0 = max |P_new|.  P0 is
    chosen far from P_new and the field anisotropic, so that normalising by
    the old iterate or by another axis' scale fails."""
    plan = schwarz.make_plan(_J3["npts"], _J3["p"], _J3["sizes"], _J3["o"])
    S = schwarz.setup(plan)
    rng = np.random.default_rng(22)
    u = [ax.u for ax in plan.axes]
    U, V, Wz = np.meshgrid(*u, indexing="ij")
    Q = np.sin(3 * U) + 0.2 * np.cos(11 * V) + 4.0 * Wz + 0.05 * rng.standard_normal(U.shape)
    P0 = 40.0 * _anisotropic(plan, rng)[::-1, ::-1, :]
    P_new, st = schwarz.sweep(S, Q, P0)
    dPs, _ = schwarz.local_corrections(S, Q, P0)
    raw = _scipy_raw_jumps(plan, dPs)
    p = plan.p
    s0 = float(np.max(np.abs(P_new)))
    sr = np.zeros((plan.dim, p))
    for a, ax in enumerate(plan.axes):
        spl = BSpline(ax.knots, P_new, p, axis=a)
        for r in range(p):
            sr[a, r] = float(np.max(np.abs((spl.derivative(r) if r else spl).c)))
    want = np.max(raw / np.maximum(sr, s0), axis=0)
    assert np.allclose(st.jump, want, rtol=1e-10, atol=0), (st.jump, want)
    # the alternatives a slip would produce all differ from it
    s0_old = float(np.max(np.abs(P0)))
    sr_old = np.zeros_like(sr)
    for a, ax in enumerate(plan.axes):
        spl = BSpline(ax.knots, P0, p, axis=a)
        for r in range(p):
            sr_old[a, r] = float(np.max(np.abs((spl.derivative(r) if r else spl).c)))
    wrong_old = np.max(raw / np.maximum(sr_old, s0_old), axis=0)
    wrong_axis = np.max(raw / np.maximum(np.roll(sr, 1, axis=0), s0), axis=0)
    wrong_nofloor = np.max(raw / sr, axis=0)
    for wrong in (wrong_old, wrong_axis):
        assert np.max(np.abs(wrong - want) / want) > 1e-3
    # the floor S_0 acts only where a derivative scale falls below max |P|
    assert np.all(sr[:, 1:] > s0) or np.any(np.abs(wrong_nofloor - want) / want > 1e-3)


def test_jump_floor_applies_when_derivative_vanishes():
    """A field constant along axis 2: its derivative coefficients along that
    axis are zero, and the floor S_0 = max |P| keeps the normalised jump
    finite and equal to raw / S_0 there."""
    plan = schwarz.make_plan(_J3["npts"], _J3["p"], _J3["sizes"], _J3["o"])
    S = schwarz.setup(plan)
    rng = np.random.default_rng(23)
    dPs = _random_local(plan, rng, 1e-6)
    base = rng.standard_normal(plan.nctrl[:2])
    P_new = np.repeat(base[:, :, None], plan.nctrl[2], axis=2)
    norm, raw = schwarz.jump_metric(S, dPs, P_new)
    s0 = float(np.max(np.abs(P_new)))
    sr2 = [float(np.max(np.abs(bspline.derivative_coefficients(P_new, plan.axes[2].knots, 3, r,
                                                                 axis=2)))) for r in (1, 2)]
    assert max(sr2) < 1e-12 * s0
    assert np.all(np.isfinite(norm))
    # axis 2 contributes raw / S_0 for r = 1, 2
    for r in (1, 2):
        assert norm[r] >= raw[2, r] / s0 * (1 - 1e-12)
