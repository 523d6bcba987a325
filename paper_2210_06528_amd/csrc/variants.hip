// Operator tables of the two model variants the paper compares with floating
// interface knots (Section 2.1; Section 3.1.1): decoupled local fits and
// clamped interfaces.  Both fits are separable, P = (L_0 x L_1 x L_2) Q, and
// so is the decode, f = (N_0 x N_1 x N_2) P, so each axis needs a fit
// operator L (control points x data points), decode rows N (one per data
// point and derivative order) and interface rows J (derivative differences of
// the two neighbours at each interface); the encode and the decode then run
// as pass chains over the axes.
#include "basis.hpp"
#include "mfa_internal.hpp"

namespace mfa {

namespace {

inline unsigned nblk(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// decoupled local fits: the free sets of the blocks side by side
// (foff[b] + local index), each fitted by its own local least-squares
// operator Z_b N[D_b, F_b]^T over the data D_b of its support.

// Fit rows: row foff[b] + j, columns D0_b .. D1_b - 1 (one workgroup per row).
__global__ void k_vdec_fit(int p, int B, const int *__restrict__ blk, const int *__restrict__ foff,
                           const int *__restrict__ span, Ell bas, const double *__restrict__ inv,
                           Ell L) {
  const int row = blockIdx.x;
  int b = 0;
  while (b + 1 < B && foff[b + 1] <= row) ++b;
  const int F0 = blk[8 * b + 2], F1 = blk[8 * b + 3], D0 = blk[8 * b + 6], D1 = blk[8 * b + 7];
  const int F = F1 - F0, j = row - foff[b];
  int64_t ioff = 0;
  for (int c = 0; c < b; ++c) {
    const int Fc = blk[8 * c + 3] - blk[8 * c + 2];
    ioff += (int64_t)Fc * Fc;
  }
  const double *Zj = inv + ioff + (int64_t)j * F;
  if (threadIdx.x == 0) L.len[row] = D1 - D0;
  for (int t = threadIdx.x; t < D1 - D0; t += blockDim.x) {
    const int i = D0 + t;
    const int s = span[i];
    double v = 0.0;
    for (int q = 0; q <= p; ++q) {
      const int k = s - p + q;
      if (k >= F0 && k < F1) v += Zj[k - F0] * bas.val[(int64_t)i * bas.L + q];
    }
    L.col[(int64_t)row * L.L + t] = i;
    L.val[(int64_t)row * L.L + t] = v;
  }
}

// Decode rows of order r = blockIdx.y: data point i takes its owner block's
// local spline (the floating-knot basis restricted to that block's free set).
__global__ void k_vdec_rows(int64_t m, int p, const int *__restrict__ blk, const int *__restrict__ foff,
                            const int *__restrict__ pown, const int *__restrict__ span, EllSet tabs,
                            EllSet out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int r = blockIdx.y;
  const Ell &src = tabs.t[r];
  const Ell &dst = out.t[r];
  const int b = pown[i];
  const int F0 = blk[8 * b + 2], F1 = blk[8 * b + 3];
  const int s = span[i];
  int len = 0;
  for (int q = 0; q <= p; ++q) {
    const int k = s - p + q;
    if (k < F0 || k >= F1) continue;
    dst.col[i * dst.L + len] = foff[b] + k - F0;
    dst.val[i * dst.L + len] = src.val[i * src.L + q];
    ++len;
  }
  dst.len[i] = len;
}

// Interface rows: row b*p + r is the r-th derivative at u*_b of block b's
// local spline minus block b+1's.
__global__ void k_vdec_jump(int nif, int p, const int *__restrict__ blk, const int *__restrict__ foff,
                            const int *__restrict__ span_if, const double *__restrict__ dbas_if,
                            Ell J) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nif * p) return;
  const int b = row / p;
  const int s = span_if[b];
  int len = 0;
  for (int side = 0; side < 2; ++side) {
    const int bb = b + side;
    const int F0 = blk[8 * bb + 2], F1 = blk[8 * bb + 3];
    for (int q = 0; q <= p; ++q) {
      const int k = s - p + q;
      if (k < F0 || k >= F1) continue;
      const double v = dbas_if[(int64_t)row * (p + 1) + q];
      J.col[(int64_t)row * J.L + len] = foff[bb] + k - F0;
      J.val[(int64_t)row * J.L + len] = side == 0 ? v : -v;
      ++len;
    }
  }
  J.len[row] = len;
}

// ---------------------------------------------------------------------------
// clamped interfaces: block b has its own clamped uniform knots with csz[b]
// control points (global columns coff[b] ..), covers the data points
// ccut[b] .. ccut[b+1] and shares its end control points with its
// neighbours.  Local parameter v = (i - ccut[b]) / (ccut[b+1] - ccut[b]),
// local span p + floor((i - ccut[b]) (nb - p) / (ccut[b+1] - ccut[b]))
// (right-continuous, the last one for v = 1).

__device__ inline int local_span(int i, int a0, int a1, int nb, int p) {
  const int64_t s = p + ((int64_t)(i - a0) * (nb - p)) / (a1 - a0);
  return (int)(s < nb - 1 ? s : nb - 1);
}

// Fit operator of block b = blockIdx.x.  Free local control points are all
// but the interface ends (lo = b > 0, hi = nb - (b < B-1)).  With G the band
// of N_free^T N_free over the block's data (factored here by one lane) and
// Z = G^-1 N_free^T, the fit of the free control points is
//   P_free = Z (y - N_left y(ccut[b]) - N_right y(ccut[b+1])),
// the interface ends taking the data at the interfaces; row j of L is Z's
// row j with -(Z N_left)_j and -(Z N_right)_j added at the two end points.
// LDS: the band (p+1) x nf and the two end corrections (2 nf).
__global__ void __launch_bounds__(256) k_vcl_fit(int p, int B, const int *__restrict__ ccut,
                                                 const int *__restrict__ coff,
                                                 const int *__restrict__ csz, Ell L, int *flag) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const int nb = csz[b], a0 = ccut[b], a1 = ccut[b + 1];
  const int nd = a1 - a0 + 1;
  const int lo = b > 0 ? 1 : 0, hi = b < B - 1 ? nb - 1 : nb;
  const int nf = hi - lo;
  double *band = lds;                        // band[t * nf + k] = G[k+t][k]
  double *cl = band + (size_t)(p + 1) * nf;  // (Z N_left)_j
  double *cr = cl + nf;                      // (Z N_right)_j
  const int row0 = coff[b] + lo;
  // band of the Gram matrix: thread per free column k; the data points in the
  // support of local function lo+k are those whose span is in [lo+k, lo+k+p]
  for (int k = threadIdx.x; k < nf; k += blockDim.x) {
    double acc[kMaxP + 1];
    for (int t = 0; t <= kMaxP; ++t) acc[t] = 0.0;
    const int fk = lo + k;
    for (int i = a0; i <= a1; ++i) {
      const int s = local_span(i, a0, a1, nb, p);
      if (s < fk || s > fk + p) continue;
      double v[kMaxP + 1];
      basis_deriv((double)(i - a0) / (double)(a1 - a0), s, nb, p, 0, v);
      const double nk = v[fk - (s - p)];
      for (int t = 0; t <= p; ++t) {
        const int fl = fk + t;
        if (fl >= hi || fl > s) break;
        acc[t] += nk * v[fl - (s - p)];
      }
    }
    for (int t = 0; t <= p; ++t) band[t * nf + k] = acc[t];
  }
  __syncthreads();
  // banded Cholesky in place (one lane): G = C C^T, lower band
  if (threadIdx.x == 0) {
    for (int j = 0; j < nf; ++j) {
      double d = band[j];
      for (int t = 1; t <= p && t <= j; ++t) {
        const double c = band[t * nf + j - t];
        d -= c * c;
      }
      if (!(d > 0.0)) {
        atomicOr(flag, 1);
        d = 1.0;
      }
      d = sqrt(d);
      band[j] = d;
      for (int t = 1; t <= p && j + t < nf; ++t) {
        double v = band[t * nf + j];
        // subtract sum_{s>=1} C[j+t][j-s] C[j][j-s]
        for (int u = 1; u + t <= p && u <= j; ++u) v -= band[(t + u) * nf + j - u] * band[u * nf + j - u];
        band[t * nf + j] = v / d;
      }
    }
  }
  __syncthreads();
  // Z column for every data point: solve G x = N_free(v_i)^T; the forward
  // sweep stores y in the table, the backward sweep overwrites it with x
  for (int t = threadIdx.x; t < nd; t += blockDim.x) {
    const int i = a0 + t;
    const int s = local_span(i, a0, a1, nb, p);
    double v[kMaxP + 1];
    basis_deriv((double)(i - a0) / (double)(a1 - a0), s, nb, p, 0, v);
    const int kmin = max(s - p - lo, 0);
    double win[kMaxP + 1];
    for (int u = 0; u <= kMaxP; ++u) win[u] = 0.0;
    for (int j = 0; j < nf; ++j) {
      double y = 0.0;
      if (j >= kmin) {
        const int fl = lo + j - (s - p);
        y = (fl >= 0 && fl <= p) ? v[fl] : 0.0;
        for (int u = 1; u <= p && u <= j; ++u) y -= band[u * nf + j - u] * win[u - 1];
        y /= band[j];
      }
      for (int u = kMaxP; u > 0; --u) win[u] = win[u - 1];
      win[0] = y;
      L.val[(int64_t)(row0 + j) * L.L + t] = y;
    }
    for (int u = 0; u <= kMaxP; ++u) win[u] = 0.0;
    for (int j = nf - 1; j >= 0; --j) {
      double x = L.val[(int64_t)(row0 + j) * L.L + t];
      for (int u = 1; u <= p && j + u < nf; ++u) x -= band[u * nf + j] * win[u - 1];
      x /= band[j];
      for (int u = kMaxP; u > 0; --u) win[u] = win[u - 1];
      win[0] = x;
      L.val[(int64_t)(row0 + j) * L.L + t] = x;
      L.col[(int64_t)(row0 + j) * L.L + t] = i;
    }
  }
  __syncthreads();
  // end corrections: (Z N_left)_j and (Z N_right)_j over the first / last span
  for (int j = threadIdx.x; j < nf; j += blockDim.x) {
    double sl = 0.0, sr = 0.0;
    for (int t = 0; t < nd; ++t) {
      const int i = a0 + t;
      const int s = local_span(i, a0, a1, nb, p);
      if (s != p && s != nb - 1) continue;
      double v[kMaxP + 1];
      basis_deriv((double)(i - a0) / (double)(a1 - a0), s, nb, p, 0, v);
      const double z = L.val[(int64_t)(row0 + j) * L.L + t];
      if (s == p) sl += z * v[0];
      if (s == nb - 1) sr += z * v[p];
    }
    cl[j] = sl;
    cr[j] = sr;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nf; j += blockDim.x) {
    if (lo == 1) L.val[(int64_t)(row0 + j) * L.L] -= cl[j];
    if (hi == nb - 1) L.val[(int64_t)(row0 + j) * L.L + nd - 1] -= cr[j];
    L.len[row0 + j] = nd;
  }
  // the interface control point after this block takes the datum there
  if (threadIdx.x == 0 && b < B - 1) {
    const int g = coff[b + 1];
    L.len[g] = 1;
    L.col[(int64_t)g * L.L] = a1;
    L.val[(int64_t)g * L.L] = 1.0;
  }
}

// Decode rows of order r = blockIdx.y (derivatives with respect to the
// physical coordinate: local v -> u -> x): point i in the owned range of
// block b (from its left interface up to its right one; the last block also
// owns m - 1).
__global__ void k_vcl_rows(int64_t m, int p, int B, const int *__restrict__ ccut,
                           const int *__restrict__ coff, const int *__restrict__ csz, double dscale,
                           EllSet out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int r = blockIdx.y;
  const Ell &dst = out.t[r];
  int b = 0;
  while (b + 1 < B && ccut[b + 1] <= i) ++b;
  const int nb = csz[b], a0 = ccut[b], a1 = ccut[b + 1];
  const int s = local_span((int)i, a0, a1, nb, p);
  double v[kMaxP + 1];
  basis_deriv((double)(i - a0) / (double)(a1 - a0), s, nb, p, r, v);
  // dv/du = (m-1)/(a1-a0), du/dx = dscale
  double sc = 1.0;
  for (int k = 0; k < r; ++k) sc *= (double)(m - 1) / (double)(a1 - a0) * dscale;
  dst.len[i] = p + 1;
  for (int q = 0; q <= p; ++q) {
    dst.col[i * dst.L + q] = coff[b] + s - p + q;
    dst.val[i * dst.L + q] = v[q] * sc;
  }
}

// Interface rows (in u): row b*p + r = d^r/du^r of block b at its right end
// minus block b+1 at its left end; gid[row] = r.
__global__ void k_vcl_jump(int64_t m, int nif, int p, const int *__restrict__ ccut,
                           const int *__restrict__ coff, const int *__restrict__ csz, Ell J,
                           int *gid) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nif * p) return;
  const int b = row / p, r = row % p;
  int len = 0;
  for (int side = 0; side < 2; ++side) {
    const int bb = b + side;
    const int nb = csz[bb], a0 = ccut[bb], a1 = ccut[bb + 1];
    const int s = side == 0 ? nb - 1 : p;
    double v[kMaxP + 1];
    basis_deriv(side == 0 ? 1.0 : 0.0, s, nb, p, r, v);
    double sc = 1.0;
    for (int k = 0; k < r; ++k) sc *= (double)(m - 1) / (double)(a1 - a0);
    for (int q = 0; q <= p; ++q) {
      J.col[(int64_t)row * J.L + len] = coff[bb] + s - p + q;
      J.val[(int64_t)row * J.L + len] = (side == 0 ? 1.0 : -1.0) * v[q] * sc;
      ++len;
    }
  }
  J.len[row] = len;
  gid[row] = r;
}

}  // namespace

#define MFA_TRY(x)                       \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

hipError_t setup_variant_axis(Handle *h, int ia, hipStream_t st) {
  Axis &X = h->ax[ia];
  const int p = h->p, B = X.B, nif = B - 1;
  const int64_t m = X.m;
  EllSet dst;
  for (int r = 0; r <= p; ++r) dst.t[r] = X.Nv[r];
  if (h->variant == MFA_VARIANT_DECOUPLED) {
    k_vdec_fit<<<(unsigned)X.nv, 256, 0, st>>>(p, B, X.d_blk, X.d_foff, X.d_span, X.N[0], X.d_inv,
                                                X.Lv);
    MFA_TRY(hipGetLastError());
    EllSet src;
    for (int r = 0; r <= p; ++r) src.t[r] = X.N[r];
    k_vdec_rows<<<dim3(nblk(m, 256), p + 1), 256, 0, st>>>(m, p, X.d_blk, X.d_foff, X.d_pown,
                                                           X.d_span, src, dst);
    MFA_TRY(hipGetLastError());
    if (nif > 0) {
      k_vdec_jump<<<nblk((int64_t)nif * p, 64), 64, 0, st>>>(nif, p, X.d_blk, X.d_foff, X.d_span_if,
                                                             X.d_dbas_if, X.Jv);
      MFA_TRY(hipGetLastError());
    }
    return hipSuccess;
  }
  if (h->variant != MFA_VARIANT_CLAMPED) return hipErrorInvalidValue;
  int nfmax = 0;
  for (int b = 0; b < B; ++b) nfmax = std::max(nfmax, X.csz[b]);
  const size_t lds = sizeof(double) * ((size_t)(p + 1) * nfmax + 2 * (size_t)nfmax);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  k_vcl_fit<<<B, 256, lds, st>>>(p, B, X.d_ccut, X.d_coff, X.d_csz, X.Lv, h->flag);
  MFA_TRY(hipGetLastError());
  k_vcl_rows<<<dim3(nblk(m, 256), p + 1), 256, 0, st>>>(m, p, B, X.d_ccut, X.d_coff, X.d_csz, X.dscale,
                                                        dst);
  MFA_TRY(hipGetLastError());
  if (nif > 0) {
    k_vcl_jump<<<nblk((int64_t)nif * p, 64), 64, 0, st>>>(m, nif, p, X.d_ccut, X.d_coff, X.d_csz, X.Jv,
                                                          X.d_gidJ);
    MFA_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace mfa
