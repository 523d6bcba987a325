// Convergence metrics of a sweep (eq. nonlinear-residuals):
//  k_deriv_scale : S_r^a = max |r-th derivative control coefficient along a|
//                  of the consensus, all axes and orders in one pass over P.
//  k_jump_expand : after the interface functional J_a has reduced axis a of the
//                  residual to (interface, order) rows, evaluate the local
//                  corrections' difference on the owned data lines of the other
//                  axes (Omega_b, Omega_c) and reduce max |.| per order.
#include "mfa_internal.hpp"

namespace mfa {

namespace {

__device__ __forceinline__ void slot_max_w(unsigned long long *slots, int slot, double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) {
    const unsigned copy = (blockIdx.x * 7u + blockIdx.y * 131u + (threadIdx.x >> 6)) % kSlotCopies;
    atomicMax(slots + (size_t)slot * kSlotCopies + copy, (unsigned long long)__double_as_longlong(v));
  }
}

struct DTab {
  const int *len;
  const int *col;
  const double *val;
  int L;
  int n;
};

// One thread per control point (grid-stride): for every active axis a and
// order r < p, the row (r, k_a) of the derivative-coefficient table applied
// along a; running maxima kept per (a, r) and reduced per wavefront.
__global__ void __launch_bounds__(256) k_deriv_scale(const double *__restrict__ P, int n0, int n1,
                                                     int n2, int p, DTab d0, DTab d1, DTab d2,
                                                     int act0, int act1, int act2,
                                                     unsigned long long *slots) {
  double mx[3][kMaxP];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int r = 0; r < kMaxP; ++r) mx[a][r] = 0.0;
  const int64_t total = (int64_t)n0 * n1 * n2;
  const int64_t s1 = n2, s0 = (int64_t)n1 * n2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k2 = (int)(i % n2);
    const int64_t t = i / n2;
    const int k1 = (int)(t % n1), k0 = (int)(t / n1);
    const int kk[3] = {k0, k1, k2};
    const int64_t st[3] = {s0, s1, 1};
    const DTab *tabs[3] = {&d0, &d1, &d2};
    const int act[3] = {act0, act1, act2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!act[a]) continue;
      const DTab &D = *tabs[a];
      int rowoff = 0;
#pragma unroll
      for (int r = 0; r < kMaxP; ++r) {
        if (r >= p) break;
        if (kk[a] <= D.n - 1 - r) {
          const int row = rowoff + kk[a];
          double s = 0.0;
          for (int q = 0; q <= r; ++q) s += D.val[(int64_t)row * D.L + q] * P[i + (int64_t)q * st[a]];
          mx[a][r] = fmax(mx[a][r], fabs(s));
        }
        rowoff += D.n - r;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int r = 0; r < kMaxP; ++r)
      if (r < p) slot_max_w(slots, kSlotS + a * kMaxP + r, mx[a][r]);
}

struct OmTab {
  const int *len;
  const int *col;
  const double *val;
  int L;
  int m;   // rows (data points)
  int n;   // columns (control points)
};

// U has shape (R, nb, nc) in the strides given (the row axis is the reduced
// interface axis; b and c are the other two axes, c may be absent with
// nc = 1).  Workgroup per (row, data point ib): V[kc] = sum_kb Om_b[ib][kb]
// U[row, kb, kc] into LDS, then every data point ic of axis c evaluates
// sum_kc Om_c[ic][kc] V[kc]; max |.| goes to slot (a, row % p).
__global__ void __launch_bounds__(256) k_jump_expand(const double *__restrict__ U, int R,
                                                     int64_t sr, int64_t sb, int64_t sc, OmTab Ob,
                                                     OmTab Oc, int has_c, int p, int slot_base,
                                                     unsigned long long *slots) {
  extern __shared__ double V[];
  const int row = blockIdx.x / Ob.m;
  const int ib = blockIdx.x % Ob.m;
  const int nc = has_c ? Oc.n : 1;
  const int lb = Ob.len[ib];
  const int *cb = Ob.col + (int64_t)ib * Ob.L;
  const double *vb = Ob.val + (int64_t)ib * Ob.L;
  for (int kc = threadIdx.x; kc < nc; kc += blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < lb; ++t) s += vb[t] * U[row * sr + (int64_t)cb[t] * sb + (int64_t)kc * sc];
    V[kc] = s;
  }
  __syncthreads();
  double mx = 0.0;
  if (has_c) {
    for (int ic = threadIdx.x; ic < Oc.m; ic += blockDim.x) {
      const int lc = Oc.len[ic];
      const int *cc = Oc.col + (int64_t)ic * Oc.L;
      const double *vc = Oc.val + (int64_t)ic * Oc.L;
      double s = 0.0;
      for (int t = 0; t < lc; ++t) s += vc[t] * V[cc[t]];
      mx = fmax(mx, fabs(s));
    }
  } else if (threadIdx.x == 0) {
    mx = fabs(V[0]);
  }
  slot_max_w(slots, slot_base + row % p, mx);
}

// 1-D: the interface rows themselves
__global__ void k_jump_rows(const double *__restrict__ U, int R, int p, int slot_base,
                            unsigned long long *slots) {
  const int r = threadIdx.x;
  const double v = r < R ? fabs(U[r]) : 0.0;
  const int slot = r < R ? slot_base + r % p : slot_base;
  // lanes name different slots: plain atomics (R is tiny)
  if (r < R)
    atomicMax(slots + (size_t)slot * kSlotCopies, (unsigned long long)__double_as_longlong(v));
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

DTab dtab(const Axis &X) { return DTab{X.D.len, X.D.col, X.D.val, X.D.L, X.n}; }
OmTab otab(const Axis &X) { return OmTab{X.Om.len, X.Om.col, X.Om.val, X.Om.L, (int)X.m, X.n}; }

}  // namespace

hipError_t launch_deriv_scale(Handle &h) {
  const int64_t total = h.nctrl_total;
  const unsigned grid = (unsigned)std::min<int64_t>(nblk(total, 256), 4096);
  k_deriv_scale<<<grid, 256, 0, h.stream>>>(h.P, h.ax[0].n, h.ax[1].n, h.ax[2].n, h.p, dtab(h.ax[0]),
                                            dtab(h.ax[1]), dtab(h.ax[2]), h.ax[0].active,
                                            h.ax[1].active, h.ax[2].active, h.slots);
  return hipGetLastError();
}

// U = J_a applied along axis a of the residual (dims with axis a of length R).
hipError_t launch_jump_expand(Handle &h, int a, const double *U) {
  const Axis &X = h.ax[a];
  const int R = (X.B - 1) * h.p;
  int64_t d[3] = {h.ax[0].n, h.ax[1].n, h.ax[2].n};
  d[a] = R;
  const int64_t st[3] = {d[1] * d[2], d[2], 1};
  int oth[2], no = 0;
  for (int c = 0; c < 3; ++c)
    if (c != a && h.ax[c].active) oth[no++] = c;
  if (no == 0) {
    k_jump_rows<<<1, 64, 0, h.stream>>>(U, R, h.p, kSlotJ + a * kMaxP, h.slots);
    return hipGetLastError();
  }
  const Axis &Xb = h.ax[oth[0]];
  const OmTab Ob = otab(Xb);
  OmTab Oc{};
  int64_t sc = 0;
  int has_c = 0;
  int nc = 1;
  if (no == 2) {
    Oc = otab(h.ax[oth[1]]);
    sc = st[oth[1]];
    has_c = 1;
    nc = h.ax[oth[1]].n;
  }
  const unsigned grid = (unsigned)((int64_t)R * Ob.m);
  k_jump_expand<<<grid, 256, sizeof(double) * nc, h.stream>>>(U, R, st[a], st[oth[0]], sc, Ob, Oc,
                                                              has_c, h.p, kSlotJ + a * kMaxP, h.slots);
  return hipGetLastError();
}

}  // namespace mfa
