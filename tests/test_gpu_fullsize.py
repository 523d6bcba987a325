"""Parity at the full 512 x 512 x 384, p = 4 size with 8 x 8 x 6 uneven
subdomains, in the configuration the benchmark times.

The oracle cannot run this size end to end in a test, so it computes sampled
outputs one by one:
  * c = N^T Q at sampled control points, each from its own support;
  * the first FP64 sweep from P = 0 at sampled control points: the combine
    (1/n_s) of the decoupled local fits of every subdomain whose free set
    holds the point, each a separable least-squares solve over that
    subdomain's data box (Algorithm 1's zero-P branch);
  * the decode at sampled grid points from the GPU's control points.
The mixed-precision encode (split-BF16 correction, FP64 residual, adaptive
checks: the benchmark's configuration) must then reach the FP64 fit within
1e-6 relative in the decoded values.
"""
import numpy as np
import pytest

from oracle import lsq, schwarz
from paper_2210_06528_amd import _lib
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def big():
    w = W.cfg_3d_mixed()
    Q = W.make_field(w)
    S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
    q = torch.from_numpy(Q).cuda()
    return w, Q, S, q


def _sample_ctrl(S, rng, count):
    """Control points at the ends, around every block's owned/free edges and at random."""
    picks = []
    for ax in S.plan.axes:
        cand = {0, ax.n - 1}
        for bl in ax.blocks:
            for k in (bl.c0, bl.c1 - 1, bl.F0, bl.F1 - 1, bl.c0 + 1):
                if 0 <= k < ax.n:
                    cand.add(k)
        picks.append(sorted(cand))
    out = []
    for _ in range(count):
        out.append(tuple(int(rng.choice(c)) if rng.random() < 0.6 else int(rng.integers(0, ax.n))
                         for c, ax in zip(picks, S.plan.axes)))
    return out


def _support(C, k):
    nz = np.nonzero(C[:, k])[0]
    return nz.min(), nz.max() + 1


def test_rhs_sampled(big):
    w, Q, S, q = big
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "fp64")
    enc.step(q)
    c = enc.inspect("rhs").reshape(w.nctrl)
    enc.close()
    rng = np.random.default_rng(11)
    Q64 = Q.astype(np.float64)
    for k in _sample_ctrl(S, rng, 60):
        rows = []
        box = []
        for a, ka in enumerate(k):
            lo, hi = _support(S.colls[a], ka)
            rows.append(S.colls[a][lo:hi, ka])
            box.append(slice(lo, hi))
        ref = np.einsum("i,j,k,ijk->", rows[0], rows[1], rows[2], Q64[tuple(box)])
        assert abs(c[k] - ref) <= 1e-12 * max(1.0, abs(ref)), (k, c[k], ref)


def test_first_sweep_sampled(big):
    w, Q, S, q = big
    enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "fp64")
    enc.step(q)
    P1 = enc.get_ctrl().cpu().numpy()
    enc.close()
    plan = S.plan
    # Z_a N_F^T of every block: the local least-squares operator of one axis
    ops = {}
    for a, ax in enumerate(plan.axes):
        for b, bl in enumerate(ax.blocks):
            NF = S.colls[a][bl.D0:bl.D1, bl.F0:bl.F1]
            ops[(a, b)] = lsq.solve_band_cholesky(S.factors[(a, b)], NF.T, axis=0)
    Q64 = Q.astype(np.float64)
    rng = np.random.default_rng(12)
    for k in _sample_ctrl(S, rng, 24):
        holders = [[b for b, bl in enumerate(ax.blocks) if bl.F0 <= k[a] < bl.F1]
                   for a, ax in enumerate(plan.axes)]
        acc, cnt = 0.0, 0
        for b0 in holders[0]:
            for b1 in holders[1]:
                for b2 in holders[2]:
                    bls = [plan.axes[a].blocks[b] for a, b in enumerate((b0, b1, b2))]
                    rows = [ops[(a, b)][k[a] - bl.F0] for a, (b, bl) in
                            enumerate(zip((b0, b1, b2), bls))]
                    box = tuple(slice(bl.D0, bl.D1) for bl in bls)
                    acc += np.einsum("i,j,k,ijk->", rows[0], rows[1], rows[2], Q64[box])
                    cnt += 1
        ref = acc / cnt
        assert abs(P1[k] - ref) <= 1e-10 * max(1.0, abs(ref)), (k, P1[k], ref)


def test_mixed_reaches_fp64_fit_and_decode_sampled(big):
    w, Q, S, q = big
    tol = w.jump_tol
    e64 = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "fp64")
    st64 = e64.encode(q, 200, tol, 0)
    assert st64["converged"]
    P64 = e64.get_ctrl().cpu().numpy()
    f64 = e64.decode(dtype=torch.float64)
    # decode at sampled grid points, evaluated by the oracle from the GPU's P
    rng = np.random.default_rng(13)
    for _ in range(40):
        i = tuple(int(rng.integers(0, m)) for m in w.npts)
        rows, box = [], []
        for a, ia in enumerate(i):
            nz = np.nonzero(S.colls[a][ia])[0]
            rows.append(S.colls[a][ia, nz.min():nz.max() + 1])
            box.append(slice(nz.min(), nz.max() + 1))
        ref = np.einsum("i,j,k,ijk->", rows[0], rows[1], rows[2], P64[tuple(box)])
        got = float(f64[i])
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (i, got, ref)
    e64.close()
    em = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, "mixed_bf16")
    stm = em.encode(q, 200, tol, 0)
    assert stm["converged"]
    fm = em.decode(dtype=torch.float32)
    err = float((fm.double() - f64).abs().max() / f64.abs().max())
    assert err < 1e-6, err
    Pm = em.get_ctrl().cpu().numpy()
    assert np.max(np.abs(Pm - P64)) / np.max(np.abs(P64)) < 1e-6
    em.close()
