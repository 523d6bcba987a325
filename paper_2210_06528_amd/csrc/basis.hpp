// Device evaluation of the basis of Section 2.1 on a clamped uniform knot
// vector: Cox-de Boor values and exact derivatives, and the rational basis of
// eq. nurbs-basis.  Shared by the setup kernels and the variant tables.
#pragma once

#include <hip/hip_runtime.h>

#include "mfa_internal.hpp"

namespace mfa {

// The decode tables of every derivative order, passed to one kernel by value.
struct EllSet {
  Ell t[kMaxP + 1];
};

// t_j of the clamped uniform knot vector: (j-p)/(n-p) clamped to [0, 1]
// (Section 2.2: clamped at the global ends, floating in the interior).
__device__ __forceinline__ double knot(int j, int n, int p) {
  const int q = j - p;
  if (q <= 0) return 0.0;
  if (q >= n - p) return 1.0;
  return (double)q / (double)(n - p);
}

// r-th derivative (r = 0: value) of the p+1 basis functions N_{s-p..s, p}
// that are nonzero in span s, at parameter u.  Degree is raised with the
// Cox-de Boor recurrence
//   N_{j,k} = (u - t_j)/(t_{j+k} - t_j) N_{j,k-1} + (t_{j+k+1} - u)/(t_{j+k+1} - t_{j+1}) N_{j+1,k-1}
// up to degree p-r, then the last r degrees use the differentiated recurrence
//   D N_{j,k} = k/(t_{j+k} - t_j) D' N_{j,k-1} - k/(t_{j+k+1} - t_{j+1}) D' N_{j+1,k-1}
// (empty knot intervals contribute nothing).  v[q] holds the function of index
// s-k+q at the current degree k.
__device__ inline void basis_deriv(double u, int s, int n, int p, int r, double *out) {
  double v[kMaxP + 1];
  double w[kMaxP + 1];
#pragma unroll
  for (int q = 0; q <= kMaxP; ++q) v[q] = 0.0;
  v[0] = 1.0;
  const int kv = p - r;
  for (int k = 1; k <= p; ++k) {
    const bool deriv = k > kv;
#pragma unroll
    for (int q = 0; q <= kMaxP; ++q) {
      if (q > k) break;
      const int j = s - k + q;
      double a = 0.0, b = 0.0;
      if (q >= 1) {
        const double tj = knot(j, n, p), tjk = knot(j + k, n, p);
        const double d = tjk - tj;
        if (d > 0.0) a = deriv ? (double)k * v[q - 1] / d : (u - tj) / d * v[q - 1];
      }
      if (q <= k - 1) {
        const double tj1 = knot(j + 1, n, p), tjk1 = knot(j + k + 1, n, p);
        const double d = tjk1 - tj1;
        if (d > 0.0) b = deriv ? (double)k * v[q] / d : (tjk1 - u) / d * v[q];
      }
      w[q] = deriv ? a - b : a + b;
    }
#pragma unroll
    for (int q = 0; q <= kMaxP; ++q)
      if (q <= k) v[q] = w[q];
  }
  for (int q = 0; q <= p; ++q) out[q] = v[q];
}

// r-th derivative of the p+1 rational basis functions R_{s-p..s} of eq.
// nurbs-basis, R_j = N_j w_j / W with W = sum_k N_k w_k, at parameter u
// (w = weights of all n control points; null: the B-spline basis).  With
// A_j = N_j w_j = W R_j, Leibniz's rule gives
//   R^(k) = (A^(k) - sum_{j=1..k} C(k, j) W^(j) R^(k-j)) / W,
// applied for k = 0..r with W^(j) = sum_q A_q^(j).
__device__ inline void basis_deriv_w(double u, int s, int n, int p, int r, const double *w, double *out) {
  if (!w) {
    basis_deriv(u, s, n, p, r, out);
    return;
  }
  double R[kMaxP + 1][kMaxP + 1];
  double Wd[kMaxP + 1];
  for (int k = 0; k <= r; ++k) {
    double a[kMaxP + 1];
    basis_deriv(u, s, n, p, k, a);
    double sum = 0.0;
    for (int q = 0; q <= p; ++q) {
      a[q] *= w[s - p + q];
      sum += a[q];
    }
    Wd[k] = sum;
    double binom = 1.0;   // C(k, j), updated as j grows
    for (int j = 1; j <= k; ++j) {
      binom = binom * (double)(k - j + 1) / (double)j;
      for (int q = 0; q <= p; ++q) a[q] -= binom * Wd[j] * R[k - j][q];
    }
    for (int q = 0; q <= p; ++q) R[k][q] = a[q] / Wd[0];
  }
  for (int q = 0; q <= p; ++q) out[q] = R[r][q];
}

}  // namespace mfa
