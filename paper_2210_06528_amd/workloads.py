"""Seeded synthetic inputs and the named workload configurations.

This module holds no part of the fitting method: it only produces data arrays
and problem descriptions (points per axis, degree, owned control points per
subdomain, overlap, stopping rule).  Both the HIP path and the CPU oracle are
fed from here, so it imports neither.

Fields
------
* 1-D:  f(x) = sin(x)/x on 2000 uniform points of [-4 pi, 4 pi].
* 2-D:  f(x, y) = sinc(x) sinc(y) + 0.1 sin(7x + 3y) on a 1024^2 grid over
        [-4 pi, 4 pi]^2, sinc(s) = sin(s)/s.
* 3-D:  a turbulent-like scalar field made of random Fourier modes with a
        k^(-5/3) amplitude spectrum and seeded phases on a periodic grid
        x_a = 2 pi i / m_a; normalised to unit RMS, stored as float32.
* The paper's own analytic test functions (the 1-D asymmetric and symmetric
  sinc sums and the 2-D/3-D radial sinc fields of Section 3) are provided for
  accuracy studies.

Grids are C-ordered with the last axis contiguous.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


def sinc(s):
    """Unnormalised sinc: sin(s)/s with sinc(0) = 1."""
    return np.sinc(np.asarray(s, dtype=np.float64) / np.pi)


# ----------------------------------------------------------------------------
# problem description
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    npts: Tuple[int, ...]            # data points per axis
    degree: int
    sizes: List[List[int]]           # owned control points per block, per axis
    overlap: int
    precision: str = "fp64"          # "fp64" | "mixed_fp32" | "mixed_bf16"
    combine: str = "avg"
    sweeps: Optional[int] = None     # fixed sweep count, or None
    jump_tol: Optional[float] = None  # stop when max_r J_r < jump_tol
    dtype: str = "f64"               # input dtype: "f64" or "f32"
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def dim(self):
        return len(self.npts)

    @property
    def nctrl(self):
        return tuple(sum(s) for s in self.sizes)

    @property
    def nsub(self):
        return tuple(len(s) for s in self.sizes)

    @property
    def npoints(self):
        return int(np.prod(self.npts))


def even_sizes(n, nb):
    """Split n control points into nb blocks whose sizes differ by at most one."""
    base, rem = divmod(n, nb)
    return [base + (1 if b < rem else 0) for b in range(nb)]


def largest_remainder(n, weights):
    """Integer sizes summing to n, proportional to weights (largest remainder)."""
    w = np.asarray(weights, dtype=np.float64)
    q = n * w / w.sum()
    base = np.floor(q).astype(np.int64)
    left = int(n - base.sum())
    order = sorted(range(len(q)), key=lambda i: (-(q[i] - base[i]), i))
    for i in order[:left]:
        base[i] += 1
    return [int(x) for x in base]


def uneven_sizes(nctrl, nsub, seed=1, spread=0.25):
    """Per-axis block sizes from weights r ~ U[1-spread, 1+spread] (one rng)."""
    rng = np.random.default_rng(seed)
    out = []
    for n, nb in zip(nctrl, nsub):
        r = rng.uniform(1.0 - spread, 1.0 + spread, nb)
        out.append(largest_remainder(n, r))
    return out


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
def field_sinc_1d(m=2000):
    x = -4.0 * np.pi + 8.0 * np.pi * np.arange(m) / (m - 1)
    return np.sin(x) / x


def field_sinc_2d(m=1024):
    x = -4.0 * np.pi + 8.0 * np.pi * np.arange(m) / (m - 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    return sinc(X) * sinc(Y) + 0.1 * np.sin(7.0 * X + 3.0 * Y)


def field_paper_1d_asymmetric(m=10000):
    """F(x) = sinc(x) + sinc(2x-1) + sinc(3x+1.5) on [-4, 4] (Section 3.1.1)."""
    x = np.linspace(-4.0, 4.0, m)
    return sinc(x) + sinc(2 * x - 1) + sinc(3 * x + 1.5)


def field_paper_1d_symmetric(m=10000):
    """F(x) = sinc(x+1) + sinc(x-1) on [-4, 4] (Section 3.1.2)."""
    x = np.linspace(-4.0, 4.0, m)
    return sinc(x + 1) + sinc(x - 1)


def field_paper_radial(shape):
    """The 2-D / 3-D radial sinc test fields of Section 3.2.3 on [-4, 4]^d."""
    axes = [np.linspace(-4.0, 4.0, m) for m in shape]
    G = np.meshgrid(*axes, indexing="ij")
    r2 = sum(g * g for g in G)
    if len(shape) == 2:
        x, y = G
        return sinc(np.sqrt(r2)) + sinc(2 * (x - 2) ** 2 + 2 * (y + 2) ** 2)
    x, y, z = G
    return sinc(np.sqrt(r2)) + sinc(2 * (x - 2) ** 2 + (y + 2) ** 2 + (z - 2) ** 2)


def _lattice_shell(dim, kmax):
    """Integer vectors with 1 <= |k| <= kmax whose first nonzero entry is > 0."""
    rng1 = np.arange(-kmax, kmax + 1)
    grids = np.meshgrid(*([rng1] * dim), indexing="ij")
    K = np.stack([g.ravel() for g in grids], axis=1)
    r2 = (K * K).sum(axis=1)
    keep = (r2 >= 1) & (r2 <= kmax * kmax)
    K = K[keep]
    first = np.zeros(len(K), dtype=np.int64)
    for a in range(dim - 1, -1, -1):
        nz = K[:, a] != 0
        first = np.where(nz, K[:, a], first)
    return K[first > 0]


def spectral_modes(dim, nmodes=512, kmax=32, seed=0):
    """Wave vectors, amplitudes |k|^(-5/3) and phases U[0, 2 pi) (one rng, in that order)."""
    rng = np.random.default_rng(seed)
    K = _lattice_shell(dim, kmax)
    pick = rng.choice(len(K), size=min(nmodes, len(K)), replace=False)
    K = K[np.sort(pick)]
    amp = np.sqrt((K * K).sum(axis=1).astype(np.float64)) ** (-5.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, len(K))
    return K, amp, phase


def field_spectral(shape, nmodes=512, kmax=32, seed=0, dtype=np.float32):
    """sum_m a_m cos(k_m . x + phi_m) on x_a = 2 pi i / m_a, unit RMS.

    Evaluated exactly (up to rounding) with one inverse real FFT of the sparse
    spectrum; every |k_a| must stay below m_a / 2.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    K, amp, phase = spectral_modes(dim, nmodes, kmax, seed)
    if np.any(np.abs(K) * 2 >= np.array(shape)[None, :]):
        raise ValueError("mode beyond the grid's Nyquist limit")
    half = shape[:-1] + (shape[-1] // 2 + 1,)
    X = np.zeros(half, dtype=np.complex128)
    coef = 0.5 * amp * np.exp(1j * phase)
    for k, c in zip(K, coef):
        if k[-1] < 0:  # cos(k.x + phi) = cos(-k.x - phi): use the half spectrum
            k, c = -k, np.conj(c)
        if k[-1] > 0:
            X[tuple(int(v) % s for v, s in zip(k, shape))] += c
        else:  # last component zero: place the conjugate pair explicitly
            X[tuple(int(v) % s for v, s in zip(k, shape))] += c
            X[tuple(int(-v) % s for v, s in zip(k, shape))] += np.conj(c)
    f = np.fft.irfftn(X, s=shape, axes=tuple(range(dim))) * float(np.prod(shape))
    f /= np.sqrt(np.mean(f * f))
    return f.astype(dtype)


def field_spectral_direct(shape, nmodes=512, kmax=32, seed=0):
    """The same field summed mode by mode (slow; for checking the FFT route)."""
    dim = len(shape)
    K, amp, phase = spectral_modes(dim, nmodes, kmax, seed)
    axes = [2.0 * np.pi * np.arange(m) / m for m in shape]
    G = np.meshgrid(*axes, indexing="ij")
    f = np.zeros(shape)
    for k, a, ph in zip(K, amp, phase):
        f += a * np.cos(sum(int(k[i]) * G[i] for i in range(dim)) + ph)
    return f / np.sqrt(np.mean(f * f))


# ----------------------------------------------------------------------------
# the named configurations
# ----------------------------------------------------------------------------
def cfg_1d():
    """1-D, FP64: sin(x)/x, 2000 points, p=3, 2 x 40 control points, overlap 3, 10 sweeps."""
    return Workload("1d-sinc-2000-p3", (2000,), 3, [[40, 40]], 3,
                    sweeps=10, dtype="f64")


def cfg_2d():
    """2-D, FP64: 1024^2 sinc field, p=3, 4x4 subdomains of 64^2 control points, overlap 2."""
    return Workload("2d-sinc-1024sq-p3", (1024, 1024), 3, [[64] * 4, [64] * 4], 2,
                    jump_tol=1e-8, dtype="f64")


def cfg_3d_batched(precision="mixed_fp32"):
    """3-D: 256^3 FP32 spectral field, p=3, 4^3 subdomains of 32^3 control points, overlap 2."""
    return Workload("3d-spectral-256cube-p3", (256, 256, 256), 3, [[32] * 4] * 3, 2,
                    precision=precision, jump_tol=1e-8, dtype="f32", seed=0)


def cfg_3d_mixed(precision="mixed_bf16"):
    """3-D: 512x512x384 FP32 spectral field, p=4, 8x8x6 uneven subdomains, overlap 2."""
    nctrl = (256, 256, 192)
    nsub = (8, 8, 6)
    return Workload("3d-spectral-512x512x384-p4-uneven", (512, 512, 384), 4,
                    uneven_sizes(nctrl, nsub, seed=1), 2,
                    precision=precision, jump_tol=1e-8, dtype="f32", seed=0)


def cfg_e1(overlap=4, m=10000, nsub=2, n_per=16):
    """1-D asymmetric sinc sum of Section 3.1.1 on [-4, 4], p=3, two subdomains."""
    w = Workload(f"e1-asym-sinc-{m}-o{overlap}", (m,), 3, [[n_per] * nsub], overlap,
                 jump_tol=1e-8, dtype="f64")
    w.extra["field"] = "e1"
    return w


def cfg_e2(nsub=5, overlap=1, m=10000, n=50):
    """1-D symmetric sinc sum of Section 3.1.2 on [-4, 4], p=3, n control points in nsub blocks."""
    w = Workload(f"e2-sym-sinc-{m}-N{nsub}-o{overlap}", (m,), 3, [even_sizes(n, nsub)], overlap,
                 jump_tol=1e-8, dtype="f64")
    w.extra["field"] = "e2"
    return w


def cfg_e5(dim=2, overlap=1):
    """Radial sinc fields of Section 3.2.3 on [-4, 4]^d: 2-D with 5x5 subdomains,
    3-D with 3x3x3, p=3, the minimum overlap (no augmented spans)."""
    if dim == 2:
        w = Workload("e5-radial-sinc-201sq", (201, 201), 3, [[12] * 5] * 2, overlap,
                     jump_tol=1e-8, dtype="f64")
    else:
        w = Workload("e5-radial-sinc-81cube", (81, 81, 81), 3, [[12] * 3] * 3, overlap,
                     jump_tol=1e-8, dtype="f64")
    w.extra["field"] = "e5"
    return w


def make_field(w: Workload):
    """The input array of a named workload (float64 or float32)."""
    kind = w.extra.get("field")
    if kind == "e1":
        return field_paper_1d_asymmetric(w.npts[0])
    if kind == "e2":
        return field_paper_1d_symmetric(w.npts[0])
    if kind == "e5":
        return field_paper_radial(w.npts)
    if w.dim == 1 and w.npts == (2000,):
        return field_sinc_1d(2000)
    if w.dim == 2 and w.npts == (1024, 1024) and w.name.startswith("2d-sinc"):
        return field_sinc_2d(1024)
    kmax = w.extra.get("kmax", 32)
    return field_spectral(w.npts, kmax=kmax, seed=w.seed,
                          dtype=np.float32 if w.dtype == "f32" else np.float64)


def small_3d(npts=(40, 36, 33), sizes=((7, 7), (6, 6), (6, 5)), p=3, overlap=2,
             precision="fp64", seed=5):
    """A small 3-D spectral workload with ragged blocks (for parity tests)."""
    w = Workload("3d-spectral-small", tuple(npts), p, [list(s) for s in sizes], overlap,
                 precision=precision, jump_tol=1e-8, dtype="f64", seed=seed)
    w.extra["kmax"] = max(1, min(npts) // 4 - 1)
    return w


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float          # seconds after stream start
    workload: Workload
    kind: str = "encode"    # "encode": a new model; "refit": new data for model `model`
    model: int = -1         # rid of the encode request that created the model
    t: float = 0.0          # time of the field (refits: the model's field advanced to t)

    def __post_init__(self):
        if self.model < 0:
            self.model = self.rid


def serving_stream(nreq=2000, rate=100.0, seed=2, side_lo=64, side_hi=512, block=32,
                   overlap=2, refit_frac=0.0, refit_window=50, refit_dt=0.02):
    """Poisson arrivals of 2-D/3-D spectral-field encode and refit requests.

    Per request (one rng, seed `seed`): inter-arrival ~ Exp(rate), dimension
    uniform in {2, 3}, sides uniform in [side_lo, side_hi], p uniform in
    {2, 3, 4}; n_a = side_a // 8 control points split into ceil(n_a / block)
    even blocks (fewer if a block would be smaller than max(p+1, 2*overlap));
    the field uses seed 1000 + rid and k_max = n_min // 4.  The rng draws do
    not depend on `rate`, so changing the rate only rescales arrival times.

    With refit_frac > 0 a second rng (seed + 1) turns that fraction of the
    requests into refits: new data for a model created by one of the last
    `refit_window` encode requests, its field advanced in time by refit_dt
    per refit (every mode's phase moves by |k| dt).  The first rng's draws
    and the arrival times are the same whatever refit_frac is.
    """
    rng = np.random.default_rng(seed)
    rrf = np.random.default_rng(seed + 1)
    t = 0.0
    out = []
    encodes = []
    nrefit = {}
    for rid in range(nreq):
        t += rng.exponential(1.0 / rate)
        dim = int(rng.integers(2, 4))
        sides = tuple(int(s) for s in rng.integers(side_lo, side_hi + 1, dim))
        p = int(rng.integers(2, 5))
        nctrl = [s // 8 for s in sides]
        # ceil(n / block) subdomains per axis, fewer where blocks would drop
        # below the minimum size max(p+1, 2*overlap)
        minb = max(p + 1, 2 * overlap)
        sizes = [even_sizes(n, max(1, min(-(-n // block), n // minb))) for n in nctrl]
        w = Workload(f"req{rid}", sides, p, sizes, overlap, precision="mixed_bf16",
                     jump_tol=1e-8, dtype="f32", seed=1000 + rid)
        w.extra["kmax"] = max(1, min(nctrl) // 4)
        if refit_frac > 0.0 and encodes and rrf.random() < refit_frac:
            cand = encodes[-refit_window:]
            m = cand[int(rrf.integers(0, len(cand)))]
            nrefit[m.rid] = nrefit.get(m.rid, 0) + 1
            out.append(Request(rid, t, m.workload, "refit", m.rid, refit_dt * nrefit[m.rid]))
            continue
        req = Request(rid, t, w, "encode", rid, 0.0)
        encodes.append(req)
        out.append(req)
    return out
