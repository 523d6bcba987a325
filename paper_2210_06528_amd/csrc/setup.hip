// Setup kernels: basis evaluation, banded normal matrices, batched banded
// Cholesky, local inverses and the per-axis operator tables.  All float64.
#include <algorithm>
#include <vector>

#include <cstring>
#include <vector>

#include "basis.hpp"
#include "mfa_internal.hpp"

namespace mfa {

namespace {

__device__ __forceinline__ int64_t dceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ int64_t d_first_with_span_ge(int s, int64_t m, int n, int p) {
  if (s <= p) return 0;
  return dceil_div((int64_t)(s - p) * (m - 1), n - p);
}

__device__ __forceinline__ int64_t d_last_with_span_le(int s, int64_t m, int n, int p) {
  if (s >= n - 1) return m - 1;
  return dceil_div((int64_t)(s - p + 1) * (m - 1), n - p) - 1;
}

// One thread per data point and derivative order r = blockIdx.y (0..p):
// span and r-th derivative basis row, written as the ELL decode table of
// that order (columns span-p..span); order 0 also writes the span.  The
// slice blockIdx.y = p + 1 evaluates the derivatives of orders 0..p-1 at the
// interface parameters u*_b (nif * p threads).

__device__ __forceinline__ void basis_rows(int64_t m, int n, int p, int *span_out, const EllSet &tabs,
                                           int nif, const double *ustar, const int *span_if,
                                           double *dbas_if, double dscale, const double *wts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int)blockIdx.y == p + 1) {
    if (i < (int64_t)nif * p) {
      const int b = (int)(i / p), r = (int)(i % p);
      basis_deriv_w(ustar[b], span_if[b], n, p, r, wts, dbas_if + i * (p + 1));
    }
    return;
  }
  if (i >= m) return;
  const int r = blockIdx.y;
  const Ell &tab = tabs.t[r];
  if (r != 0) span_out = nullptr;
  int64_t s = p + (i * (n - p)) / (m - 1);
  if (s > n - 1) s = n - 1;
  const double u = (double)i / (double)(m - 1);
  double vals[kMaxP + 1];
  basis_deriv_w(u, (int)s, n, p, r, wts, vals);
  // derivative rows with respect to the physical coordinate (du/dx)^r
  double sc = 1.0;
  for (int k = 0; k < r; ++k) sc *= dscale;
  if (span_out) span_out[i] = (int)s;
  tab.len[i] = p + 1;
  for (int q = 0; q <= p; ++q) {
    tab.col[i * tab.L + q] = (int)s - p + q;
    tab.val[i * tab.L + q] = r == 0 ? vals[q] : vals[q] * sc;
  }
}


// Banded normal matrix A = N^T N of one axis, lower band storage
// band[t*n + k] = A[k+t][k].  One wavefront per row k: the lanes stride over
// the data points in the support of N_k and the p+1 partial sums are reduced
// across the wavefront with shuffles (fixed order, deterministic).
__device__ __forceinline__ void gram_row(int64_t m, int n, int p, const int *span, const Ell &basis,
                                         double *band) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  const int smin = max(k, p), smax = min(k + p, n - 1);
  const int64_t lo = d_first_with_span_ge(smin, m, n, p);
  const int64_t hi = d_last_with_span_le(smax, m, n, p);
  double acc[kMaxP + 1];
#pragma unroll
  for (int t = 0; t <= kMaxP; ++t) acc[t] = 0.0;
  for (int64_t i = lo + lane; i <= hi; i += 64) {
    const int s = span[i];
    const double *b = basis.val + i * basis.L;
    const double nk = b[k - s + p];
#pragma unroll
    for (int t = 0; t <= kMaxP; ++t)
      if (t <= p && k + t <= s) acc[t] += nk * b[k + t - s + p];
  }
#pragma unroll
  for (int t = 0; t <= kMaxP; ++t) {
    double v = acc[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[t] = v;
  }
  if (lane == 0)
    for (int t = 0; t <= p; ++t) band[(int64_t)t * n + k] = (k + t < n) ? acc[t] : 0.0;
}

// Batched banded Cholesky of every subdomain's local normal matrix
// A[F0:F1, F0:F1] (a principal block of the axis' band; Section 2.3.1), for
// degree PP.  A wavefront per matrix stages the block's band in LDS (entries
// past the block read as zero); one lane then forms the columns in order,
// keeping the last PP columns of L in registers, so a column costs a square
// root, a division and O(PP^2) register products with no LDS round trip on
// its chain.  A non-positive pivot sets flag[0].
template <int PP>
__global__ void __launch_bounds__(64) k_chol(int n, const double *band, const int *blk,
                                             double *chol, double *rdiag, int *flag) {
  extern __shared__ double As[];   // As[t*F + j] = A(j+t, j)
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  int64_t off = 0, roff = 0;
  for (int bb = 0; bb < b; ++bb) {
    off += (int64_t)(PP + 1) * (blk[8 * bb + 3] - blk[8 * bb + 2]);
    roff += blk[8 * bb + 3] - blk[8 * bb + 2];
  }
  const int F0 = blk[8 * b + 2], F = blk[8 * b + 3] - F0;
  for (int e = lane; e < (PP + 1) * F; e += 64) {
    const int t = e / F, j = e - t * F;
    As[e] = j + t < F ? band[(int64_t)t * n + F0 + j] : 0.0;
  }
  __syncthreads();
  if (lane != 0) return;
  // cl[q][t] = L(j-1-q+t, j-1-q): the PP columns before column j (zero
  // before column 0 and below row F-1)
  double cl[PP][PP + 1];
#pragma unroll
  for (int q = 0; q < PP; ++q)
#pragma unroll
    for (int t = 0; t <= PP; ++t) cl[q][t] = 0.0;
  double a[PP + 1];
#pragma unroll
  for (int t = 0; t <= PP; ++t) a[t] = As[t * F];
  for (int j = 0; j < F; ++j) {
    double an[PP + 1];
    const int jn = min(j + 1, F - 1);
#pragma unroll
    for (int t = 0; t <= PP; ++t) an[t] = As[t * F + jn];
    // pivot: A(j,j) - sum_k L(j,k)^2 over k = j-PP .. j-1 in increasing k
    const double ajj = a[0];
    double d = ajj;
#pragma unroll
    for (int q = PP - 1; q >= 0; --q) d -= cl[q][q + 1] * cl[q][q + 1];
    if (!(d > 1e-13 * ajj) || !(d > 0.0)) {
      atomicOr(flag, 1);
      d = 1.0;
    }
    const double ljj = sqrt(d);
    // L(j+t, j) = (A(j+t, j) - sum_k L(j+t,k) L(j,k)) / L(j,j)
    double nw[PP + 1];
    nw[0] = ljj;
#pragma unroll
    for (int t = 1; t <= PP; ++t) {
      double s = a[t];
#pragma unroll
      for (int q = PP - 1 - t; q >= 0; --q) s -= cl[q][q + 1 + t] * cl[q][q + 1];
      nw[t] = s / ljj;
    }
#pragma unroll
    for (int t = 0; t <= PP; ++t) chol[off + (int64_t)t * F + j] = nw[t];
    rdiag[roff + j] = 1.0 / ljj;
#pragma unroll
    for (int q = PP - 1; q > 0; --q)
#pragma unroll
      for (int t = 0; t <= PP; ++t) cl[q][t] = cl[q - 1][t];
#pragma unroll
    for (int t = 0; t <= PP; ++t) {
      cl[0][t] = nw[t];
      a[t] = an[t];
    }
  }
}

// The same with the factor in global memory (segments too long for LDS).
__global__ void __launch_bounds__(64) k_chol_global(int n, int p, const double *band, const int *blk,
                                             double *chol, double *rdiag, int *flag) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  int64_t off = 0, roff = 0;
  for (int bb = 0; bb < b; ++bb) {
    off += (int64_t)(p + 1) * (blk[8 * bb + 3] - blk[8 * bb + 2]);
    roff += blk[8 * bb + 3] - blk[8 * bb + 2];
  }
  const int F0 = blk[8 * b + 2], F = blk[8 * b + 3] - F0;
  double *L = chol + off;  // L[t*F + j] = L(j+t, j)
  for (int j = 0; j < F; ++j) {
    if (lane == 0) {
      const double ajj = band[F0 + j];
      double s = ajj;
      for (int k = max(0, j - p); k < j; ++k) {
        const double l = L[(j - k) * F + k];
        s -= l * l;
      }
      if (!(s > 1e-13 * ajj) || !(s > 0.0)) {
        atomicOr(flag, 1);
        s = 1.0;
      }
      L[j] = sqrt(s);
      rdiag[roff + j] = 1.0 / L[j];
    }
    __syncthreads();
    if (lane >= 1 && lane <= p) {
      const int i = j + lane;
      if (i < F) {
        double s = band[(int64_t)lane * n + F0 + j];
        for (int k = max(0, i - p); k < j; ++k) s -= L[(i - k) * F + k] * L[(j - k) * F + k];
        L[lane * F + j] = s / L[j];
      } else {
        L[lane * F + j] = 0.0;
      }
    }
    __syncthreads();
  }
}

// Dense inverse of every local normal matrix from its banded Cholesky factor:
// column `col` solves L L^T z = e_col by forward and backward substitution.
__global__ void k_inverse_global(int p, const int *blk, const double *chol, double *inv) {
  const int b = blockIdx.x;
  int64_t offc = 0, offi = 0;
  for (int bb = 0; bb < b; ++bb) {
    const int Fb = blk[8 * bb + 3] - blk[8 * bb + 2];
    offc += (int64_t)(p + 1) * Fb;
    offi += (int64_t)Fb * Fb;
  }
  const int F = blk[8 * b + 3] - blk[8 * b + 2];
  const double *L = chol + offc;
  double *Z = inv + offi;
  for (int col = threadIdx.x; col < F; col += blockDim.x) {
    for (int i = 0; i < F; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      if (i > col)
        for (int k = max(col, i - p); k < i; ++k) s -= L[(i - k) * F + k] * Z[(int64_t)k * F + col];
      Z[(int64_t)i * F + col] = (i < col) ? 0.0 : s / L[i];
    }
    for (int i = F - 1; i >= 0; --i) {
      double s = Z[(int64_t)i * F + col];
      for (int k = i + 1; k <= min(F - 1, i + p); ++k) s -= L[(k - i) * F + i] * Z[(int64_t)k * F + col];
      Z[(int64_t)i * F + col] = s / L[i];
    }
  }
}

// The same with the factor and the inverse in LDS (F^2 + (p+1)F doubles),
// written out coalesced at the end.
// Factor and dense inverse of every local normal matrix in one launch, for
// degree PP, when both fit in LDS.  Lane 0 forms the banded Cholesky factor
// column by column as k_chol does (last PP columns in registers), writing it
// in place over the staged band in LDS and out to chol/rdiag; then a thread
// per column solves L L^T z = e_col from LDS.  Each substitution keeps the
// last PP values of its column in registers (zero before the column's first
// nonzero, and the factor's band padding is zero, so every term is formed
// without a branch) and adds the newest one last, so a step waits on a
// single product of the step before; the diagonal is applied as a
// reciprocal.  A non-positive pivot sets flag[0].
template <int PP>
__device__ __forceinline__ void chol_inv_block(int n, const double *band, const int *blk, double *chol,
                                               double *rdiag, double *inv, int *flag) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  int64_t off = 0, roff = 0, offi = 0;
  for (int bb = 0; bb < b; ++bb) {
    const int Fb = blk[8 * bb + 3] - blk[8 * bb + 2];
    off += (int64_t)(PP + 1) * Fb;
    roff += Fb;
    offi += (int64_t)Fb * Fb;
  }
  const int F0 = blk[8 * b + 2], F = blk[8 * b + 3] - F0;
  double *L = sm;                            // [(PP+1) * F]: A(j+t, j), then L(j+t, j)
  double *Z = sm + (size_t)(PP + 1) * F;     // [F * F]
  double *rL = Z + (size_t)F * F;            // [F], 1 / L(i, i)
  for (int e = threadIdx.x; e < (PP + 1) * F; e += blockDim.x) {
    const int t = e / F, j = e - t * F;
    L[e] = j + t < F ? band[(int64_t)t * n + F0 + j] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // cl[q][t] = L(j-1-q+t, j-1-q): the PP columns before column j
    double cl[PP][PP + 1];
#pragma unroll
    for (int q = 0; q < PP; ++q)
#pragma unroll
      for (int t = 0; t <= PP; ++t) cl[q][t] = 0.0;
    double a[PP + 1];
#pragma unroll
    for (int t = 0; t <= PP; ++t) a[t] = L[t * F];
    for (int j = 0; j < F; ++j) {
      double an[PP + 1];
      const int jn = min(j + 1, F - 1);
#pragma unroll
      for (int t = 0; t <= PP; ++t) an[t] = L[t * F + jn];
      const double ajj = a[0];
      double d = ajj;
#pragma unroll
      for (int q = PP - 1; q >= 0; --q) d -= cl[q][q + 1] * cl[q][q + 1];
      if (!(d > 1e-13 * ajj) || !(d > 0.0)) {
        atomicOr(flag, 1);
        d = 1.0;
      }
      const double ljj = sqrt(d);
      double nw[PP + 1];
      nw[0] = ljj;
#pragma unroll
      for (int t = 1; t <= PP; ++t) {
        double s = a[t];
#pragma unroll
        for (int q = PP - 1 - t; q >= 0; --q) s -= cl[q][q + 1 + t] * cl[q][q + 1];
        nw[t] = s / ljj;
      }
      // column j of A has been read (into a); column j+1 is in an
#pragma unroll
      for (int t = 0; t <= PP; ++t) {
        L[t * F + j] = nw[t];
        chol[off + (int64_t)t * F + j] = nw[t];
      }
      rdiag[roff + j] = 1.0 / ljj;
#pragma unroll
      for (int q = PP - 1; q > 0; --q)
#pragma unroll
        for (int t = 0; t <= PP; ++t) cl[q][t] = cl[q - 1][t];
#pragma unroll
      for (int t = 0; t <= PP; ++t) {
        cl[0][t] = nw[t];
        a[t] = an[t];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < F; e += blockDim.x) rL[e] = 1.0 / L[e];
  __syncthreads();
  for (int col = threadIdx.x; col < F; col += blockDim.x) {
    // forward: z = L^{-1} e_col, w[r] = z_{i-1-r} (zero before col); the
    // factor entries read for i - 1 - r < 0 lie inside L and meet a zero
    double w[PP];
#pragma unroll
    for (int r = 0; r < PP; ++r) w[r] = 0.0;
    for (int i = 0; i < col; ++i) Z[i * F + col] = 0.0;
    for (int i = col; i < F; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
#pragma unroll
      for (int r = PP - 1; r >= 0; --r) s -= L[(r + 1) * F + i - 1 - r] * w[r];
      const double z = s * rL[i];
#pragma unroll
      for (int r = PP - 1; r > 0; --r) w[r] = w[r - 1];
      w[0] = z;
      Z[i * F + col] = z;
    }
    // backward: x = L^{-T} z, w[r] = x_{i+1+r} (zero past F, where the
    // factor's padding L(i+1+r, i) is zero too)
#pragma unroll
    for (int r = 0; r < PP; ++r) w[r] = 0.0;
    for (int i = F - 1; i >= 0; --i) {
      double s = Z[i * F + col];
#pragma unroll
      for (int r = PP - 1; r >= 0; --r) s -= L[(r + 1) * F + i] * w[r];
      const double x = s * rL[i];
#pragma unroll
      for (int r = PP - 1; r > 0; --r) w[r] = w[r - 1];
      w[0] = x;
      Z[i * F + col] = x;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < F * F; e += blockDim.x) inv[offi + e] = Z[e];
}

__device__ __forceinline__ int64_t inv_offset(const int *blk, int b) {
  int64_t off = 0;
  for (int bb = 0; bb < b; ++bb) {
    const int Fb = blk[8 * bb + 3] - blk[8 * bb + 2];
    off += (int64_t)Fb * Fb;
  }
  return off;
}

__device__ __forceinline__ void pad_row(Ell &t, int64_t r, int len) {
  t.len[r] = len;
  const int last = len > 0 ? t.col[r * t.L + len - 1] : 0;
  for (int q = len; q < t.L; ++q) {
    t.col[r * t.L + q] = last;
    t.val[r * t.L + q] = 0.0;
  }
  if (t.valf)
    for (int q = 0; q < t.L; ++q) t.valf[r * t.L + q] = (float)t.val[r * t.L + q];
}

// N^T: row k lists the data points whose span lies in [k, k+p].
__device__ __forceinline__ void tab_NT(int64_t m, int n, int p, const int *span, Ell basis, Ell t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t lo = d_first_with_span_ge(max(k, p), m, n, p);
  const int64_t hi = d_last_with_span_le(min(k + p, n - 1), m, n, p);
  int len = 0;
  for (int64_t i = lo; i <= hi; ++i, ++len) {
    const int s = span[i];
    t.col[(int64_t)k * t.L + len] = (int)i;
    t.val[(int64_t)k * t.L + len] = basis.val[i * basis.L + (k - s + p)];
  }
  pad_row(t, k, len);
}

// A = N^T N as rows: columns k-p..k+p from the band.
__device__ __forceinline__ void tab_A(int n, int p, const double *band, Ell t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int len = 0;
  for (int c = max(0, k - p); c <= min(n - 1, k + p); ++c, ++len) {
    const int lo = min(k, c), d = abs(k - c);
    t.col[(int64_t)k * t.L + len] = c;
    t.val[(int64_t)k * t.L + len] = band[(int64_t)d * n + lo];
  }
  pad_row(t, k, len);
}

// Weighted additive-Schwarz operator of one axis:
// M[k][:] = sum over blocks b whose free set holds k of w_k Z_b[k - F0_b][:],
// w_k = 1/n_s(k) (combine AVG) or the owner indicator (combine RAS).
__device__ __forceinline__ void tab_M(int n, int combine, const int *blk, const int *blo,
                                              const int *bhi, const int *owner, const int *ns,
                                              const double *inv, Ell t) {
  // one wavefront per row, lanes over its columns (each entry written once)
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  int b0 = blo[k], b1 = bhi[k];
  if (combine == MFA_COMBINE_RAS) b0 = b1 = owner[k];
  const int cfirst = blk[8 * b0 + 2], clast = blk[8 * b1 + 3];
  const double w = combine == MFA_COMBINE_RAS ? 1.0 : 1.0 / (double)ns[k];
  const int len = clast - cfirst;
  for (int q = lane; q < t.L; q += 64) {
    const int col = cfirst + q;
    double v = 0.0;
    if (q < len) {
      for (int b = b0; b <= b1; ++b) {
        const int F0 = blk[8 * b + 2], F = blk[8 * b + 3] - F0;
        if (col >= F0 && col < F0 + F) v += w * inv[inv_offset(blk, b) + (int64_t)(k - F0) * F + (col - F0)];
      }
    }
    t.col[(int64_t)k * t.L + q] = q < len ? col : (len > 0 ? clast - 1 : 0);
    t.val[(int64_t)k * t.L + q] = v;
  }
  if (lane == 0) t.len[k] = len;
}

// Decode of a subdomain's local correction at its owned data points:
// Om[i][:] = sum_q N_{s-p+q}(u_i) Z_b[s-p+q - F0_b][:] over the free set of the
// block b that owns point i (basis functions outside F_b carry no correction).
__device__ __forceinline__ void tab_Om(int64_t m, int p, const int *blk, const int *pown,
                                               const int *span, Ell basis, const double *inv, Ell t,
                                               double *valT) {
  // one wavefront per data point, lanes over the free set of its owner
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = pown[i];
  const int F0 = blk[8 * b + 2], F = blk[8 * b + 3] - F0;
  const double *Z = inv + inv_offset(blk, b);
  const int s = span[i];
  for (int c = lane; c < t.L; c += 64) {
    double acc = 0.0;
    if (c < F) {
      for (int q = 0; q <= p; ++q) {
        const int j = s - p + q - F0;
        if (j >= 0 && j < F) acc += basis.val[i * basis.L + q] * Z[(int64_t)j * F + c];
      }
    }
    t.col[i * t.L + c] = c < F ? F0 + c : F0 + F - 1;
    t.val[i * t.L + c] = acc;
    valT[(int64_t)c * m + i] = acc;   // the values transposed: valT[c*m + i]
  }
  if (lane == 0) t.len[i] = F;
}

// Interface jump functionals: row (b, r) maps a residual line to
// d^r/du^r (L_b - L_{b+1})(u*_b) = dB_r(u*)^T (E_b Z_b R_b - E_{b+1} Z_{b+1} R_{b+1}).
__device__ __forceinline__ void tab_J(int nif, int p, const int *blk, const int *span_if,
                                              const double *dbas, const double *inv, Ell t, int *gid) {
  // one wavefront per row (b, r), lanes over its columns
  const int row = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = row / p, r = row % p;
  const int cfirst = blk[8 * b + 2], clast = blk[8 * (b + 1) + 3];
  const int len = clast - cfirst;
  const double *dv = dbas + (int64_t)row * (p + 1);
  const int s = span_if[b];
  for (int q = lane; q < t.L; q += 64) {
    const int col = cfirst + q;
    double v = 0.0;
    if (q < len) {
      for (int side = 0; side < 2; ++side) {
        const int bb = b + side;
        const double sgn = side == 0 ? 1.0 : -1.0;
        const int F0 = blk[8 * bb + 2], F = blk[8 * bb + 3] - F0;
        if (col < F0 || col >= F0 + F) continue;
        const double *Z = inv + inv_offset(blk, bb);
        for (int qq = 0; qq <= p; ++qq) {
          const int j = s - p + qq - F0;
          if (j < 0 || j >= F) continue;
          v += sgn * dv[qq] * Z[(int64_t)j * F + (col - F0)];
        }
      }
    }
    t.col[(int64_t)row * t.L + q] = q < len ? col : (len > 0 ? clast - 1 : 0);
    t.val[(int64_t)row * t.L + q] = v;
  }
  if (lane == 0) {
    t.len[row] = len;
    gid[row] = r;
  }
}

// Derivative-coefficient operator: rows of D^r for r = 0..p-1 stacked; row k
// of D^r gives the r-th derivative control coefficient
//   D^r_k = (p-r+1)/(t_{k+p+1} - t_{k+r}) (D^{r-1}_{k+1} - D^{r-1}_k),  D^0 = P.
__device__ __forceinline__ void tab_D(int n, int p, Ell t, int *gid) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  int r = 0, base = 0;
  while (r < p && row >= base + (n - r)) {
    base += n - r;
    ++r;
  }
  if (r >= p) return;
  const int k = row - base;
  // c[l][i]: coefficients (over P_{k..k+r}) of D^l_{k+i}
  double c[kMaxP + 1][kMaxP + 1];
  for (int i = 0; i <= r; ++i)
    for (int q = 0; q <= r; ++q) c[i][q] = (i == q) ? 1.0 : 0.0;
  for (int l = 1; l <= r; ++l) {
    for (int i = 0; i <= r - l; ++i) {
      const int kk = k + i;
      const double den = knot(kk + p + 1, n, p) - knot(kk + l, n, p);
      const double f = den > 0.0 ? (double)(p - l + 1) / den : 0.0;
      for (int q = 0; q <= r; ++q) c[i][q] = f * (c[i + 1][q] - c[i][q]);
    }
  }
  for (int q = 0; q <= r; ++q) {
    t.col[(int64_t)row * t.L + q] = k + q;
    t.val[(int64_t)row * t.L + q] = c[0][q];
  }
  pad_row(t, row, r + 1);
  gid[row] = r;
}

// ----------------------------------------------------------------- DATABOX
// segmented decode: row (b, i) for data point i of D_b (rows of N gathered)
__global__ void k_tab_Nseg(int p, int B, const int *blk, const int64_t *doff_unused, Ell basis,
                           Ell t, int *qmap) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= t.R) return;
  int b = 0;
  int64_t base = 0;
  while (b < B) {
    const int64_t nd = (int64_t)blk[8 * b + 7] - blk[8 * b + 6];
    if (row < base + nd) break;
    base += nd;
    ++b;
  }
  const int64_t i = blk[8 * b + 6] + (row - base);
  qmap[row] = (int)i;
  for (int q = 0; q <= p; ++q) {
    t.col[row * t.L + q] = basis.col[i * basis.L + q];
    t.val[row * t.L + q] = basis.val[i * basis.L + q];
  }
  pad_row(t, row, p + 1);
}

// segmented N_F^T: row (b, k), k in F_b, over the segment of D_b
__global__ void k_tab_NsegT(int64_t m, int n, int p, int B, const int *blk, const int *span,
                            Ell basis, Ell t) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= t.R) return;
  int b = 0;
  int64_t base = 0, dbase = 0;
  while (b < B) {
    const int64_t nf = (int64_t)blk[8 * b + 3] - blk[8 * b + 2];
    if (row < base + nf) break;
    base += nf;
    dbase += (int64_t)blk[8 * b + 7] - blk[8 * b + 6];
    ++b;
  }
  const int k = blk[8 * b + 2] + (int)(row - base);
  int64_t lo = d_first_with_span_ge(max(k, p), m, n, p);
  int64_t hi = d_last_with_span_le(min(k + p, n - 1), m, n, p);
  const int64_t D0 = blk[8 * b + 6], D1 = blk[8 * b + 7];
  lo = lo > D0 ? lo : D0;
  hi = hi < D1 - 1 ? hi : D1 - 1;
  int len = 0;
  for (int64_t i = lo; i <= hi; ++i, ++len) {
    const int s = span[i];
    t.col[row * t.L + len] = (int)(dbase + (i - D0));
    t.val[row * t.L + len] = basis.val[i * basis.L + (k - s + p)];
  }
  pad_row(t, row, len);
}

// interface functional on the segmented free layout: row (b, r) has the
// Z_b part on segment b and the -Z_{b+1} part on segment b+1
__global__ void k_tab_Jseg(int nif, int p, const int *blk, const int *span_if, const double *dbas,
                           const double *inv, Ell t) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nif * p) return;
  const int b = row / p;
  const double *dv = dbas + (int64_t)row * (p + 1);
  const int s = span_if[b];
  int len = 0;
  for (int side = 0; side < 2; ++side) {
    const int bb = b + side;
    const double sgn = side == 0 ? 1.0 : -1.0;
    int64_t base = 0;
    for (int q = 0; q < bb; ++q) base += blk[8 * q + 3] - blk[8 * q + 2];
    const int F0 = blk[8 * bb + 2], F = blk[8 * bb + 3] - F0;
    const double *Z = inv + inv_offset(blk, bb);
    for (int c = 0; c < F; ++c) {
      double v = 0.0;
      for (int q = 0; q <= p; ++q) {
        const int j = s - p + q - F0;
        if (j >= 0 && j < F) v += dv[q] * Z[(int64_t)j * F + c];
      }
      t.col[(int64_t)row * t.L + len] = (int)(base + c);
      t.val[(int64_t)row * t.L + len] = sgn * v;
      ++len;
    }
  }
  pad_row(t, row, len);
}

// owned-data decode of the local correction on the segmented free layout
__global__ void k_tab_Omseg(int64_t m, const int *blk, const int *pown, Ell om, Ell t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int b = pown[i];
  int64_t base = 0;
  for (int q = 0; q < b; ++q) base += blk[8 * q + 3] - blk[8 * q + 2];
  const int F0 = blk[8 * b + 2];
  const int len = om.len[i];
  for (int c = 0; c < len; ++c) {
    t.col[i * t.L + c] = (int)(base + (om.col[i * om.L + c] - F0));
    t.val[i * t.L + c] = om.val[i * om.L + c];
  }
  pad_row(t, i, len);
}

// block-diagonal local inverse on the segmented free layout
__global__ void k_tab_Zseg(int B, const int *blk, const double *inv, Ell t) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= t.R) return;
  int b = 0;
  int64_t base = 0;
  while (b < B) {
    const int64_t nf = (int64_t)blk[8 * b + 3] - blk[8 * b + 2];
    if (row < base + nf) break;
    base += nf;
    ++b;
  }
  const int F = blk[8 * b + 3] - blk[8 * b + 2];
  const int j = (int)(row - base);
  const double *Z = inv + inv_offset(blk, b);
  for (int c = 0; c < F; ++c) {
    t.col[row * t.L + c] = (int)(base + c);
    t.val[row * t.L + c] = Z[(int64_t)j * F + c];
  }
  pad_row(t, row, F);
}

// combine from the segmented free layout back to the control grid
__global__ void k_tab_Comb(int n, int combine, const int *blk, const int *blo, const int *bhi,
                           const int *owner, const int *ns, Ell t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int b0 = blo[k], b1 = bhi[k];
  if (combine == MFA_COMBINE_RAS) b0 = b1 = owner[k];
  const double w = combine == MFA_COMBINE_RAS ? 1.0 : 1.0 / (double)ns[k];
  int len = 0;
  for (int b = b0; b <= b1; ++b) {
    int64_t base = 0;
    for (int bb = 0; bb < b; ++bb) base += blk[8 * bb + 3] - blk[8 * bb + 2];
    t.col[(int64_t)k * t.L + len] = (int)(base + (k - blk[8 * b + 2]));
    t.val[(int64_t)k * t.L + len] = w;
    ++len;
  }
  pad_row(t, k, len);
}


// stencil rows: acoef[k*(2p+1) + t] = A[k][k-p+t], zero outside the matrix
__device__ __forceinline__ void tab_acoef(int n, int p, const double *band, double *acoef) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  for (int t = 0; t <= 2 * p; ++t) {
    const int c = k - p + t;
    double v = 0.0;
    if (c >= 0 && c < n) v = band[(int64_t)abs(k - c) * n + min(k, c)];
    acoef[(int64_t)k * (2 * p + 1) + t] = v;
  }
}

// The row tables that need only the basis rows and the normal-matrix band,
// in one launch (a thread per row, blockIdx.y the table): N^T, A, the
// derivative operators D and the residual stencil rows.
__device__ __forceinline__ void tab_rows(int64_t m, int n, int p, const int *span, const Ell &basis,
                                         const Ell &NT, const double *band, const Ell &A, const Ell &D,
                                         int *gidD, double *acoef) {
  switch (blockIdx.y) {
    case 0: tab_NT(m, n, p, span, basis, NT); break;
    case 1: tab_A(n, p, band, A); break;
    case 2: tab_D(n, p, D, gidD); break;
    default: tab_acoef(n, p, band, acoef); break;
  }
}

// The operators built from the local inverses, in one launch (a wavefront
// per row, blockIdx.y the table): M (n rows), Om (m data points, with its
// values also written transposed) and the interface functionals J (nif * p
// rows, none with one block).
__device__ __forceinline__ void tab_ops(int64_t m, int n, int p, int combine, int nif, const int *blk,
                                        const int *blo, const int *bhi, const int *owner, const int *ns,
                                        const int *pown, const int *span, const Ell &basis,
                                        const double *inv, const int *span_if, const double *dbas_if,
                                        const Ell &M, const Ell &Om, double *omT, const Ell &J,
                                        int *gidJ) {
  switch (blockIdx.y) {
    case 0:
      if (blockIdx.x < (unsigned)n) tab_M(n, combine, blk, blo, bhi, owner, ns, inv, M);
      break;
    case 1:
      if (blockIdx.x < (uint64_t)m) tab_Om(m, p, blk, pown, span, basis, inv, Om, omT);
      break;
    default:
      if (blockIdx.x < (unsigned)(nif * p)) tab_J(nif, p, blk, span_if, dbas_if, inv, J, gidJ);
      break;
  }
}

// Setup stages of every active axis in one launch each: blockIdx.z selects
// the axis, whose arguments travel in a small array (the grid covers the
// largest axis; every stage checks its own bounds).  One launch per stage
// instead of one per stage and axis: setup is bound by the host's launch
// rate, not by these kernels.
template <typename A>
struct Tri {
  A a[3];
};

struct BasisArgs {
  int64_t m;
  int n, p, nif;
  int *span;
  EllSet tabs;
  const double *ustar;
  const int *span_if;
  double *dbas_if;
  double dscale;
  const double *w;
};

struct GramArgs {
  int64_t m;
  int n, p;
  const int *span;
  Ell basis;
  double *band;
};

struct RowsArgs {
  int64_t m;
  int n, p;
  const int *span;
  Ell basis, NT, A, D;
  const double *band;
  int *gidD;
  double *acoef;
};

struct CholArgs {
  int n, B;
  const double *band;
  const int *blk;
  double *chol, *rdiag, *inv;
};

struct OpsArgs {
  int64_t m;
  int n, p, nif;
  const int *blk, *blo, *bhi, *owner, *ns, *pown, *span, *span_if;
  Ell basis, M, Om, J;
  const double *inv, *dbas_if;
  double *omT;
  int *gidJ;
};

__global__ void k_basis3(Tri<BasisArgs> t) {
  const BasisArgs &a = t.a[blockIdx.z];
  basis_rows(a.m, a.n, a.p, a.span, a.tabs, a.nif, a.ustar, a.span_if, a.dbas_if, a.dscale, a.w);
}

__global__ void __launch_bounds__(64) k_gram3(Tri<GramArgs> t) {
  const GramArgs &a = t.a[blockIdx.z];
  if (blockIdx.x >= (unsigned)a.n) return;
  gram_row(a.m, a.n, a.p, a.span, a.basis, a.band);
}

__global__ void k_tab_rows3(Tri<RowsArgs> t) {
  const RowsArgs &a = t.a[blockIdx.z];
  tab_rows(a.m, a.n, a.p, a.span, a.basis, a.NT, a.band, a.A, a.D, a.gidD, a.acoef);
}

template <int PP>
__global__ void __launch_bounds__(256) k_chol_inv3(Tri<CholArgs> t, int *flag) {
  const CholArgs &a = t.a[blockIdx.z];
  if (blockIdx.x >= (unsigned)a.B) return;   // whole workgroups, before any barrier
  chol_inv_block<PP>(a.n, a.band, a.blk, a.chol, a.rdiag, a.inv, flag);
}

__global__ void __launch_bounds__(64) k_tab_ops3(Tri<OpsArgs> t, int combine) {
  const OpsArgs &a = t.a[blockIdx.z];
  tab_ops(a.m, a.n, a.p, combine, a.nif, a.blk, a.blo, a.bhi, a.owner, a.ns, a.pown, a.span, a.basis,
          a.inv, a.span_if, a.dbas_if, a.M, a.Om, a.omT, a.J, a.gidJ);
}

// Decode at arbitrary points: one thread per point, the p+1 basis values
// (or derivatives) per active axis from the Cox-de Boor recurrence, then the
// (p+1)^d tensor sum over the control points under the point's spans.
struct PtAxes {
  int n[3], active[3], ua[3], r[3];
  const double *w[3];   // NURBS weights per axis (null: B-spline)
  double scale;         // product of (du/dx)^r over the axes
};

template <typename TO>
__global__ void k_decode_points(const double *__restrict__ u, int64_t npts, int dim, int p, PtAxes ax,
                                const double *__restrict__ P, TO *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  double val[3][kMaxP + 1];
  int s0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!ax.active[a]) {
      s0[a] = 0;
      val[a][0] = 1.0;
      continue;
    }
    const int n = ax.n[a];
    double x = u[i * dim + ax.ua[a]];
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    int s = p + (int)floor(x * (double)(n - p));
    s = s < p ? p : (s > n - 1 ? n - 1 : s);
    // largest s in [p, n-1] with t_s <= x (right-continuous, as on the grid)
    while (s > p && knot(s, n, p) > x) --s;
    while (s < n - 1 && knot(s + 1, n, p) <= x) ++s;
    basis_deriv_w(x, s, n, p, ax.r[a], ax.w[a], val[a]);
    s0[a] = s - p;
  }
  const int w0 = ax.active[0] ? p + 1 : 1, w1 = ax.active[1] ? p + 1 : 1, w2 = ax.active[2] ? p + 1 : 1;
  const int64_t n1 = ax.n[1], n2 = ax.n[2];
  double acc = 0.0;
  for (int q0 = 0; q0 < w0; ++q0)
    for (int q1 = 0; q1 < w1; ++q1) {
      const double v01 = val[0][q0] * val[1][q1];
      const double *row = P + ((int64_t)(s0[0] + q0) * n1 + (s0[1] + q1)) * n2 + s0[2];
      double t = 0.0;
      for (int q2 = 0; q2 < w2; ++q2) t += val[2][q2] * row[q2];
      acc += v01 * t;
    }
  out[i] = (TO)(acc * ax.scale);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace


#define MFA_TRY(x)                       \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

hipError_t upload_plan(Handle *h, std::vector<char> &img) {
  img.assign(h->upload_bytes, 0);
  auto put = [&](void *dev, const void *src, size_t bytes) {
    if (bytes) std::memcpy(img.data() + ((char *)dev - h->ws), src, bytes);
  };
  const int p = h->p;
  if (h->variant == MFA_VARIANT_CLAMPED) {
    for (int ia = 0; ia < 3; ++ia) {
      Axis &X = h->ax[ia];
      if (!X.active) continue;
      put(X.d_ccut, X.ccut.data(), sizeof(int) * X.ccut.size());
      put(X.d_coff, X.coff.data(), sizeof(int) * X.coff.size());
      put(X.d_csz, X.csz.data(), sizeof(int) * X.csz.size());
    }
    if (img.empty()) return hipSuccess;
    return hipMemcpyAsync(h->ws, img.data(), img.size(), hipMemcpyHostToDevice, h->stream);
  }
  for (int ia = 0; ia < 3; ++ia) {
    Axis &X = h->ax[ia];
    if (!X.active) {
      std::vector<double> id((size_t)(2 * p + 1) * X.n, 0.0);
      for (int k = 0; k < X.n; ++k) id[(size_t)k * (2 * p + 1) + p] = 1.0;
      put(X.d_acoef, id.data(), sizeof(double) * id.size());
      continue;
    }
    const int n = X.n, B = X.B, nif = B - 1;
    std::vector<int> blk(8 * B), choff(B), foff(B);
    for (int b = 0; b < B; ++b) {
      const Block &Bk = X.blk[b];
      int *e = &blk[8 * b];
      e[0] = Bk.c0; e[1] = Bk.c1; e[2] = Bk.F0; e[3] = Bk.F1;
      e[4] = (int)Bk.own0; e[5] = (int)Bk.own1; e[6] = (int)Bk.D0; e[7] = (int)Bk.D1;
      choff[b] = (int)X.chol_off[b];
      foff[b] = (int)X.foff[b];
    }
    put(X.d_blk, blk.data(), sizeof(int) * blk.size());
    put(X.d_blo, X.blo.data(), sizeof(int) * n);
    put(X.d_bhi, X.bhi.data(), sizeof(int) * n);
    put(X.d_owner, X.owner.data(), sizeof(int) * n);
    put(X.d_ns, X.ns.data(), sizeof(int) * n);
    put(X.d_pown, X.pown.data(), sizeof(int) * X.m);
    put(X.d_choff, choff.data(), sizeof(int) * B);
    put(X.d_foff, foff.data(), sizeof(int) * B);
    if (nif > 0) {
      put(X.d_ustar, X.ustar.data(), sizeof(double) * nif);
      put(X.d_span_if, X.span_if.data(), sizeof(int) * nif);
    }
    if (X.d_w) put(X.d_w, X.w.data(), sizeof(double) * n);
  }
  // the caller keeps the image until its next synchronisation of the stream
  return hipMemcpyAsync(h->ws, img.data(), img.size(), hipMemcpyHostToDevice, h->stream);
}

hipError_t setup_axes(Handle *h, hipStream_t st) {
  const int p = h->p;
  int act[3], na = 0;
  for (int a = 0; a < 3; ++a)
    if (h->ax[a].active) act[na++] = a;
  if (na == 0) return hipSuccess;
  Tri<BasisArgs> tb{};
  Tri<GramArgs> tg{};
  Tri<RowsArgs> tr{};
  Tri<OpsArgs> to{};
  unsigned gb = 1, gg = 1, gr = 1, go = 1;
  bool any_if = false;
  for (int k = 0; k < na; ++k) {
    Axis &X = h->ax[act[k]];
    const int n = X.n, nif = X.B - 1;
    const int64_t m = X.m;
    X.d_bas = X.N[0].val;
    BasisArgs &b = tb.a[k];
    b.m = m;
    b.n = n;
    b.p = p;
    b.nif = nif;
    b.span = X.d_span;
    for (int r = 0; r <= p; ++r) b.tabs.t[r] = X.N[r];
    b.ustar = X.d_ustar;
    b.span_if = X.d_span_if;
    b.dbas_if = X.d_dbas_if;
    b.dscale = X.dscale;
    b.w = X.d_w;
    gb = std::max(gb, nblk(std::max<int64_t>(m, (int64_t)nif * p), 256));
    tg.a[k] = GramArgs{m, n, p, X.d_span, X.N[0], X.d_gram};
    gg = std::max<unsigned>(gg, (unsigned)n);
    RowsArgs &rw = tr.a[k];
    rw.m = m;
    rw.n = n;
    rw.p = p;
    rw.span = X.d_span;
    rw.basis = X.N[0];
    rw.NT = X.NT;
    rw.A = X.A;
    rw.D = X.D;
    rw.band = X.d_gram;
    rw.gidD = X.d_gidD;
    rw.acoef = X.d_acoef;
    gr = std::max(gr, nblk(std::max<int64_t>(n, X.ND), 128));
    OpsArgs &o = to.a[k];
    o.m = m;
    o.n = n;
    o.p = p;
    o.nif = nif;
    o.blk = X.d_blk;
    o.blo = X.d_blo;
    o.bhi = X.d_bhi;
    o.owner = X.d_owner;
    o.ns = X.d_ns;
    o.pown = X.d_pown;
    o.span = X.d_span;
    o.span_if = X.d_span_if;
    o.basis = X.N[0];
    o.M = X.M;
    o.Om = X.Om;
    o.J = X.J;
    o.inv = X.d_inv;
    o.dbas_if = X.d_dbas_if;
    o.omT = X.d_omT;
    o.gidJ = X.d_gidJ;
    go = std::max<unsigned>(go, (unsigned)std::max<int64_t>(std::max<int64_t>(n, m), (int64_t)nif * p));
    any_if = any_if || nif > 0;
  }
  // basis values and derivative tables at the data points, all orders
  k_basis3<<<dim3(gb, any_if ? p + 2 : p + 1, na), 256, 0, st>>>(tb);
  MFA_TRY(hipGetLastError());
  k_gram3<<<dim3(gg, 1, na), 64, 0, st>>>(tg);
  MFA_TRY(hipGetLastError());
  // N^T, A, D and the stencil rows (they need the basis rows and the band)
  k_tab_rows3<<<dim3(gr, 4, na), 128, 0, st>>>(tr);
  MFA_TRY(hipGetLastError());
  // factor and local inverses: one launch for the axes whose blocks fit in
  // LDS together with their inverses; the others take the factor (LDS or
  // global) and the inverses from global memory
  Tri<CholArgs> tc{};
  int nc = 0;
  unsigned gc = 1;
  size_t clds = 0;
  for (int k = 0; k < na; ++k) {
    Axis &X = h->ax[act[k]];
    const size_t chol_lds = sizeof(double) * (p + 1) * X.Fmax;
    const size_t inv_lds = sizeof(double) * ((size_t)(p + 2) * X.Fmax + (size_t)X.Fmax * X.Fmax);
    if (inv_lds <= 64 * 1024 && p >= 1 && p <= 8) {
      tc.a[nc++] = CholArgs{X.n, X.B, X.d_gram, X.d_blk, X.d_chol, X.d_rdiag, X.d_inv};
      gc = std::max<unsigned>(gc, (unsigned)X.B);
      clds = std::max(clds, inv_lds);
      continue;
    }
    if (chol_lds <= 64 * 1024 && p >= 1 && p <= 8) {
      switch (p) {
#define MFA_CHOL_CASE(PP)                                                                            \
  case PP:                                                                                           \
    k_chol<PP><<<X.B, 64, chol_lds, st>>>(X.n, X.d_gram, X.d_blk, X.d_chol, X.d_rdiag, h->flag); \
    break;
        MFA_CHOL_CASE(1)
        MFA_CHOL_CASE(2)
        MFA_CHOL_CASE(3)
        MFA_CHOL_CASE(4)
        MFA_CHOL_CASE(5)
        MFA_CHOL_CASE(6)
        MFA_CHOL_CASE(7)
        MFA_CHOL_CASE(8)
#undef MFA_CHOL_CASE
        default:
          break;
      }
    } else {
      k_chol_global<<<X.B, 64, 0, st>>>(X.n, p, X.d_gram, X.d_blk, X.d_chol, X.d_rdiag, h->flag);
    }
    MFA_TRY(hipGetLastError());
    k_inverse_global<<<X.B, 256, 0, st>>>(p, X.d_blk, X.d_chol, X.d_inv);
    MFA_TRY(hipGetLastError());
  }
  if (nc > 0) {
    switch (p) {
#define MFA_CHOLINV_CASE(PP)                                                        \
  case PP:                                                                          \
    k_chol_inv3<PP><<<dim3(gc, 1, nc), 256, clds, st>>>(tc, h->flag);               \
    break;
      MFA_CHOLINV_CASE(1)
      MFA_CHOLINV_CASE(2)
      MFA_CHOLINV_CASE(3)
      MFA_CHOLINV_CASE(4)
      MFA_CHOLINV_CASE(5)
      MFA_CHOLINV_CASE(6)
      MFA_CHOLINV_CASE(7)
      MFA_CHOLINV_CASE(8)
#undef MFA_CHOLINV_CASE
      default:
        break;
    }
    MFA_TRY(hipGetLastError());
  }
  // M, Om and J (they need the local inverses)
  k_tab_ops3<<<dim3(go, any_if ? 3 : 2, na), 64, 0, st>>>(to, h->combine);
  MFA_TRY(hipGetLastError());
  if (h->rhs == MFA_RHS_DATABOX) {
    for (int k = 0; k < na; ++k) {
      Axis &X = h->ax[act[k]];
      const int n = X.n, B = X.B, nif = B - 1;
      const int64_t m = X.m;
      k_tab_Nseg<<<nblk(X.SD, 128), 128, 0, st>>>(p, B, X.d_blk, nullptr, X.N[0], X.Nseg, X.d_qmap);
      k_tab_NsegT<<<nblk(X.SF, 128), 128, 0, st>>>(m, n, p, B, X.d_blk, X.d_span, X.N[0], X.NsegT);
      k_tab_Zseg<<<nblk(X.SF, 64), 64, 0, st>>>(B, X.d_blk, X.d_inv, X.Zseg);
      k_tab_Comb<<<nblk(n, 128), 128, 0, st>>>(n, h->combine, X.d_blk, X.d_blo, X.d_bhi, X.d_owner,
                                               X.d_ns, X.Comb);
      if (nif > 0)
        k_tab_Jseg<<<nblk((int64_t)nif * p, 64), 64, 0, st>>>(nif, p, X.d_blk, X.d_span_if, X.d_dbas_if,
                                                              X.d_inv, X.Jseg);
      k_tab_Omseg<<<nblk(m, 128), 128, 0, st>>>(m, X.d_blk, X.d_pown, X.Om, X.Omseg);
      MFA_TRY(hipGetLastError());
    }
  }
  return hipSuccess;
}


hipError_t launch_decode_points(Handle &h, const double *u, int64_t npts, void *out, bool f32,
                                const int r[3]) {
  if (npts == 0) return hipSuccess;
  PtAxes ax{};
  ax.scale = 1.0;
  for (int a = 0; a < 3; ++a) {
    ax.n[a] = h.ax[a].n;
    ax.active[a] = h.ax[a].active;
    ax.ua[a] = a - (3 - h.dim);
    ax.r[a] = r[a];
    ax.w[a] = h.ax[a].d_w;
    for (int k = 0; k < r[a]; ++k) ax.scale *= h.ax[a].dscale;
  }
  const unsigned grid = (unsigned)((npts + 255) / 256);
  if (f32)
    k_decode_points<float><<<grid, 256, 0, h.stream>>>(u, npts, h.dim, h.p, ax, h.P, (float *)out);
  else
    k_decode_points<double><<<grid, 256, 0, h.stream>>>(u, npts, h.dim, h.p, ax, h.P, (double *)out);
  return hipGetLastError();
}

}  // namespace mfa
