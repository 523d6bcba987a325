// Convergence metrics of a sweep (eq. nonlinear-residuals):
//  k_deriv_scale : S_r^a = max |r-th derivative control coefficient along a|
//                  of the consensus, all axes and orders in one pass over P.
//  k_jump_project: the interface functionals J_a (all orders of an interface
//                  at once) applied along axis a of the residual.
//  k_jump_expand : after the interface functional J_a has reduced axis a of the
//                  residual to (interface, order) rows, evaluate the local
//                  corrections' difference on the owned data lines of the other
//                  axes (Omega_b, Omega_c) and reduce max |.| per order.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

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

// The workgroup's max of v, one atomic on one copy of the slot (wavefront
// maxima through LDS, then thread 0); every thread must call it.  One atomic
// per workgroup instead of one per wavefront: the atomics on a slot's copies
// queue at L2, a tail for kernels whose workgroups all finish together.
__device__ __forceinline__ void block_slot_max_w(unsigned long long *slots, int slot, double v) {
  __shared__ double red[16];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < nw; ++i) m = fmax(m, red[i]);
    const unsigned copy = (blockIdx.x * 7u + blockIdx.y * 131u + blockIdx.z * 1031u) % kSlotCopies;
    atomicMax(slots + (size_t)slot * kSlotCopies + copy, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ double tod(double v) { return v; }
__device__ __forceinline__ double tod(float v) { return (double)v; }
__device__ __forceinline__ double tod(__hip_bfloat16 v) { return (double)__bfloat162float(v); }


struct DTab {
  const int *len;
  const int *col;
  const double *val;
  int L;
  int n;
};

struct OmTab {
  const int *len;
  const int *col;
  const double *val;
  const double *valT;   // val transposed: valT[t*m + i] = val[i*L + t]
  int L;
  int m;   // rows (data points)
  int n;   // columns (control points)
};

// U has shape (R, nb, nc) in the strides given (the row axis is the reduced
// interface axis; b and c are the other two axes, c may be absent with
// nc = 1).  Workgroup per (row, group of `jb` data points ib):
// V_i[kc] = sum_kb Om_b[ib_i][kb] U[row, kb, kc] into LDS, then every data
// point ic of axis c evaluates sum_kc Om_c[ic][kc] V_i[kc] for all i of the
// group (one read of the Om_c row serves jb outputs); max |.| goes to slot
// (a, row % p).  Om rows are contiguous column ranges (the free set of the
// point's owner), so the group's rows are laid out densely over the union
// of their ranges (at most wmax columns, from the host): a thread per kc
// then reads each U value of that range once and feeds all jb sums, the row
// coefficients being the same for the whole wavefront (LDS broadcasts).
template <int JB>
__global__ void __launch_bounds__(256) k_jump_expand(const double *__restrict__ U, int R,
                                                     int64_t sr, int64_t sb, int64_t sc, OmTab Ob,
                                                     OmTab Oc, int has_c, int p, int slot_base,
                                                     unsigned long long *slots, int wmax) {
  constexpr int jb = JB;
  extern __shared__ double V[];   // [jb][nc]
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that
  // each XCD takes a contiguous run of rows and their U rows stay in that
  // XCD's L2 (a bijection on [0, gridDim.x)).
  const unsigned G = gridDim.x, xcd = blockIdx.x % 8, per = G / 8, rem = G % 8;
  const unsigned lb = xcd * per + min(xcd, rem) + blockIdx.x / 8;
  const int nbg = (Ob.m + jb - 1) / jb;
  const int row = lb / nbg;
  const int ib0 = (lb % nbg) * jb;
  const int nib = min(jb, Ob.m - ib0);
  const int nc = has_c ? Oc.n : 1;
  // the group's Om_b rows, dense over the union [kb0, kb0 + W) of their ranges
  double *VB = V + jb * nc;                                   // [jb][wmax]
  int *CB = reinterpret_cast<int *>(VB + jb * wmax);          // [jb][2]: start, length
  for (int i = threadIdx.x; i < jb; i += blockDim.x) {
    CB[2 * i] = i < nib ? Ob.col[(int64_t)(ib0 + i) * Ob.L] : 0;
    CB[2 * i + 1] = i < nib ? Ob.len[ib0 + i] : 0;
  }
  __syncthreads();
  int kb0 = CB[0], kb1 = CB[0] + CB[1];
  for (int i = 1; i < nib; ++i) {
    kb0 = min(kb0, CB[2 * i]);
    kb1 = max(kb1, CB[2 * i] + CB[2 * i + 1]);
  }
  const int W = min(kb1 - kb0, wmax);   // the host sizes wmax to the widest union
  for (int e = threadIdx.x; e < jb * wmax; e += blockDim.x) {
    const int i = e / wmax, t = e - i * wmax;
    const int q = kb0 + t - CB[2 * i];
    VB[e] = (i < nib && t < W && q >= 0 && q < CB[2 * i + 1]) ? Ob.val[(int64_t)(ib0 + i) * Ob.L + q] : 0.0;
  }
  __syncthreads();
  for (int kc = threadIdx.x; kc < nc; kc += blockDim.x) {
    double acc[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) acc[i] = 0.0;
    const double *u = U + row * sr + (int64_t)kb0 * sb + (int64_t)kc * sc;
    // eight strided loads in flight per step
    for (int t0 = 0; t0 < W; t0 += 8) {
      double x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = t0 + q < W ? u[(int64_t)(t0 + q) * sb] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int t = min(t0 + q, wmax - 1);
#pragma unroll
        for (int i = 0; i < JB; ++i) acc[i] += VB[i * wmax + t] * x[q];
      }
    }
#pragma unroll
    for (int i = 0; i < JB; ++i) V[i * nc + kc] = acc[i];
  }
  __syncthreads();
  double mx = 0.0;
  if (has_c) {
    for (int ic = threadIdx.x; ic < Oc.m; ic += blockDim.x) {
      const int lc = Oc.len[ic];
      const int cc0 = Oc.col[(int64_t)ic * Oc.L];
      const double *vc = Oc.valT + ic;
      const double *vrow = V + cc0;
      double acc[JB];
#pragma unroll
      for (int i = 0; i < JB; ++i) acc[i] = 0.0;
      // coefficients read eight at a time so their loads overlap
      for (int t0 = 0; t0 < lc; t0 += 8) {
        double wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) wv[u] = t0 + u < lc ? vc[(int64_t)(t0 + u) * Oc.m] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (t0 + u < lc) {
#pragma unroll
            for (int i = 0; i < JB; ++i) acc[i] += wv[u] * vrow[i * nc + t0 + u];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < JB; ++i)
        if (i < nib) mx = fmax(mx, fabs(acc[i]));
    }
  } else {
    for (int i = threadIdx.x; i < nib; i += blockDim.x) mx = fmax(mx, fabs(V[i]));
  }
  block_slot_max_w(slots, slot_base + row % p, mx);
}

// 1-D: the interface rows themselves
__global__ void k_jump_rows(const double *__restrict__ U, int R, int p, int slot_base,
                            unsigned long long *slots) {
  // lanes name different slots: plain atomics (R is tiny)
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    atomicMax(slots + (size_t)(slot_base + r % p) * kSlotCopies,
              (unsigned long long)__double_as_longlong(fabs(U[r])));
}

// U[..., b*p + r, ...] = sum_k J[b*p + r][k] g[..., k, ...] for every
// interface b of axis a and order r < p (all orders from one read of the
// interface's support); U has the layout of g with axis a replaced by the
// (B-1)*p interface rows.  Grid: (ceil(n2'/bs), n1', n0') over U's dims with
// axis a collapsed to the interface index.
template <typename TG>
__global__ void __launch_bounds__(256) k_jump_project(const TG *__restrict__ g, double *__restrict__ U,
                                                      int a, int n0, int n1, int n2, int nif, int p,
                                                      const int *__restrict__ Jcol,
                                                      const int *__restrict__ Jlen,
                                                      const double *__restrict__ Jval, int LJ) {
  extern __shared__ double sJ[];   // the workgroup's interface rows [p][LJ]
  // output coordinates with axis a replaced by the interface index b (uniform
  // over the workgroup: grid.z for a = 0, grid.y for a = 1)
  int d[3] = {n0, n1, n2};
  d[a] = nif;
  const int x2 = blockIdx.x * blockDim.x + threadIdx.x;
  int x[3] = {(int)blockIdx.z, (int)blockIdx.y, x2};
  const int b = x[a];
  const int row0 = b * p;
  for (int e = threadIdx.x; e < p * LJ; e += blockDim.x) sJ[e] = Jval[(int64_t)row0 * LJ + e];
  __syncthreads();
  if (x2 >= d[2]) return;
  const int64_t gs[3] = {(int64_t)n1 * n2, n2, 1};
  int R[3] = {n0, n1, n2};
  R[a] = nif * p;
  const int64_t us[3] = {(int64_t)R[1] * R[2], R[2], 1};
  x[a] = 0;
  const int64_t gbase = x[0] * gs[0] + x[1] * gs[1] + x[2] * gs[2];
  const int64_t ubase = x[0] * us[0] + x[1] * us[1] + x[2] * us[2];
  const int c0 = Jcol[(int64_t)row0 * LJ];
  const int len = Jlen[row0];
  const TG *src = g + gbase + (int64_t)c0 * gs[a];
  double acc[kMaxP];
#pragma unroll
  for (int r = 0; r < kMaxP; ++r) acc[r] = 0.0;
  // eight strided loads in flight per step
  for (int t0 = 0; t0 < len; t0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = t0 + u < len ? tod(src[(int64_t)(t0 + u) * gs[a]]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (t0 + u < len) {
#pragma unroll
        for (int r = 0; r < kMaxP; ++r)
          if (r < p) acc[r] += sJ[r * LJ + t0 + u] * v[u];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kMaxP; ++r)
    if (r < p) U[ubase + (int64_t)(row0 + r) * us[a]] = acc[r];
}

// S_r^a for all axes and orders, one workgroup per grid row (x0, x1) with the
// lanes over axis 2: the coefficient rows of axes 0 and 1 are uniform over the
// workgroup; those of axis 2 are per lane (a small table, cache resident).
__global__ void __launch_bounds__(256) k_deriv_scale(const double *__restrict__ P, int n0, int n1,
                                                     int n2, int p, DTab d0, DTab d1, DTab d2,
                                                     int act0, int act1, int act2, int rows,
                                                     unsigned long long *slots) {
  const int k2 = blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.z;
  const bool valid = k2 < n2;
  const int64_t st[3] = {(int64_t)n1 * n2, n2, 1};
  const DTab *tabs[3] = {&d0, &d1, &d2};
  const int act[3] = {act0, act1, act2};
  double mx[3][kMaxP];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int r = 0; r < kMaxP; ++r) mx[a][r] = 0.0;
  const int k1lo = blockIdx.y * rows, k1hi = min(n1, k1lo + rows);
  for (int k1 = k1lo; k1 < k1hi; ++k1) {
    const int64_t i = ((int64_t)k0 * n1 + k1) * n2 + (valid ? k2 : 0);
    const int kk[3] = {k0, k1, k2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!act[a]) continue;
      const DTab &D = *tabs[a];
      int rowoff = 0;
#pragma unroll
      for (int r = 0; r < kMaxP; ++r) {
        if (r >= p) break;
        if (valid && kk[a] <= D.n - 1 - r) {
          const double *dv = D.val + (int64_t)(rowoff + kk[a]) * D.L;
          double s = 0.0;
          for (int q = 0; q <= r; ++q) s += dv[q] * P[i + (int64_t)q * st[a]];
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
      if (act[a] && r < p) slot_max_w(slots, kSlotS + a * kMaxP + r, mx[a][r]);
}

// Interface projection along the contiguous axis: one lane per grid line
// (x0, x1), all interfaces and orders.
template <typename TG>
__global__ void __launch_bounds__(256) k_jump_project_inner(const TG *__restrict__ g,
                                                            double *__restrict__ U, int64_t nlines,
                                                            int n2, int nif, int p,
                                                            const int *__restrict__ Jcol,
                                                            const int *__restrict__ Jlen,
                                                            const double *__restrict__ Jval, int LJ) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  const int b = blockIdx.y;
  const TG *src = g + l * n2;
  const int row0 = b * p;
  const int c0 = Jcol[(int64_t)row0 * LJ];
  const int len = Jlen[row0];
  double acc[kMaxP];
#pragma unroll
  for (int r = 0; r < kMaxP; ++r) acc[r] = 0.0;
  for (int t = 0; t < len; ++t) {
    const double v = tod(src[c0 + t]);
#pragma unroll
    for (int r = 0; r < kMaxP; ++r)
      if (r < p) acc[r] += Jval[(int64_t)(row0 + r) * LJ + t] * v;
  }
#pragma unroll
  for (int r = 0; r < kMaxP; ++r)
    if (r < p) U[(int64_t)(row0 + r) * nlines + l] = acc[r];
}

// Interface projection along the contiguous axis: a workgroup stages LPB
// whole grid lines of g in LDS (one coalesced read) and computes every
// (line, interface) pair, all orders from one pass over the interface's
// support.  The lines are staged in SG, float for a float or BF16 residual
// (its values exactly) and double otherwise.
template <typename TG, typename SG>
__global__ void __launch_bounds__(256) k_jump_project_lines(const TG *__restrict__ g,
                                                            double *__restrict__ U, int64_t nlines,
                                                            int n2, int nif, int p, int LPB,
                                                            const int *__restrict__ Jcol,
                                                            const int *__restrict__ Jlen,
                                                            const double *__restrict__ Jval, int LJ) {
  extern __shared__ double smem_j[];
  double *sJ = smem_j;                                  // the J rows [nif*p][LJ]
  SG *sg = reinterpret_cast<SG *>(sJ + (size_t)nif * p * LJ);   // [LPB][ldg]
  // staged lines ldg = n2 | 1 elements apart: the lanes of a wave read the
  // same column of consecutive lines, which an even line length (n2 = 192:
  // a multiple of the 32 banks) would put all in one LDS bank
  const int ldg = n2 | 1;
  const int64_t l0 = (int64_t)blockIdx.x * LPB;
  const int nl = (int)min((int64_t)LPB, nlines - l0);
  for (int e = threadIdx.x; e < nif * p * LJ; e += blockDim.x) sJ[e] = Jval[e];
  const TG *src = g + l0 * n2;
  // 16 loads per thread in flight before the first store
  for (int e0 = 0; e0 < nl * n2; e0 += blockDim.x * 16) {
    SG v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + threadIdx.x + blockDim.x * u;
      v[u] = e < nl * n2 ? (SG)tod(src[e]) : SG(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + threadIdx.x + blockDim.x * u;
      if (e < nl * n2) {
        const int li = e / n2;
        sg[li * ldg + (e - li * n2)] = v[u];
      }
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < nl * nif; it += blockDim.x) {
    const int b = it / nl, li = it - b * nl;
    const int row0 = b * p;
    const int c0 = Jcol[(int64_t)row0 * LJ];
    const int len = Jlen[row0];
    const SG *x = sg + li * ldg + c0;
    double acc[kMaxP];
#pragma unroll
    for (int r = 0; r < kMaxP; ++r) acc[r] = 0.0;
    const double *jr = sJ + (size_t)row0 * LJ;
    // eight terms per step: their LDS reads are issued before the first use
    for (int t0 = 0; t0 < len; t0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = t0 + u < len ? x[t0 + u] : 0.0;
#pragma unroll
      for (int r = 0; r < kMaxP; ++r) {
        if (r < p) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (t0 + u < len) acc[r] += jr[r * LJ + t0 + u] * v[u];
        }
      }
    }
    // U[row][line]: the interface rows outermost (coalesced here and in the
    // expansion, whose lanes run along the contiguous other axis)
#pragma unroll
    for (int r = 0; r < kMaxP; ++r)
      if (r < p) U[(int64_t)(row0 + r) * nlines + l0 + li] = acc[r];
  }
}

// Interface projection on the matrix cores (FP64 MFMA, v_mfma_f64_16x16x4_f64):
// U[row][col] = sum_k J[row][k] g[k][col], where k runs along axis a and col
// over the other coordinates (their layout in strides: g element (k, col) at
// gbase + k*gsk + col*gsc, U element (row, col) at ubase + row*usk + col),
// with an outer index o for the axis-1 case (a line of axis 2 per o).  A wave
// forms one 16 x 16 tile (16 interface rows, 16 columns): the K range is the
// union of its rows' supports, and K-step s pairs operand slot q with
// k = k0 + 4q + s, so that for the contiguous axis (CONTIG: columns are lines
// of g, k contiguous) a lane's four values of four consecutive steps are one
// 16-byte load.  Lane layout, checked by an in-bounds probe: A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k, and D[i][j] in lane j + 16(i%4),
// register i/4 (the FP32 instruction's D differs: lane j + 16(i/4), register
// i%4).  A = J (rows from the table), B = g, D = U.  J rows outside their
// support and columns past the array contribute zero.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename TG, bool CONTIG>
__global__ void __launch_bounds__(256) k_jproj_mfma(const TG *__restrict__ g, double *__restrict__ U, int R,
                                                    int nrt, int64_t ncol, int nct, int64_t gstride_o,
                                                    int64_t ustride_o, int64_t gsk, int64_t gsc, int64_t usk,
                                                    int nk, int64_t ntask, const int *__restrict__ Jcol,
                                                    const int *__restrict__ Jlen,
                                                    const double *__restrict__ Jval, int LJ) {
  const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t task = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (task >= ntask) return;   // whole waves
  const int T = (int)(task % nrt);
  const int64_t ctg = task / nrt;
  const int64_t o = ctg / nct;
  const int64_t col = (ctg % nct) * 16 + c;
  const bool colok = col < ncol;
  const TG *gb = g + o * gstride_o + (colok ? col : 0) * gsc;
  // this lane's J row (as operand row c) and the tile's K range
  const int row = 16 * T + c;
  const bool rowok = row < R;
  const int c0 = rowok ? Jcol[(int64_t)row * LJ] : (1 << 30);
  const int len = rowok ? Jlen[row] : 0;
  int klo = rowok ? c0 : (1 << 30), khi = rowok ? c0 + len : 0;
  for (int off = 32; off > 0; off >>= 1) {
    klo = min(klo, __shfl_xor(klo, off, 64));
    khi = max(khi, __shfl_xor(khi, off, 64));
  }
  klo = __builtin_amdgcn_readfirstlane(klo) & ~3;
  khi = __builtin_amdgcn_readfirstlane(khi);
  const double *jr = Jval + (int64_t)(rowok ? row : 0) * LJ;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  // J operands of the four consecutive k from k4 (zero outside the row)
  auto load_a = [&](int k4, double (&a)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int t = k4 + s - c0;
      a[s] = (t >= 0 && t < len) ? jr[t] : 0.0;
    }
  };
  // residual operands: k4 .. k4+3 of this lane's column (zero past the axis
  // or the columns); one 16-byte read when they are contiguous floats
  const bool vec = CONTIG && sizeof(TG) == 4 && (nk & 3) == 0 && (gsc & 3) == 0;
  auto load_b = [&](int k4, double (&b)[4]) {
    if (vec && k4 + 3 < nk) {
      const float4 f = *reinterpret_cast<const float4 *>(gb + k4);
      b[0] = colok ? f.x : 0.0;
      b[1] = colok ? f.y : 0.0;
      b[2] = colok ? f.z : 0.0;
      b[3] = colok ? f.w : 0.0;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = min(k4 + s, nk - 1);
        const double v = tod(gb[(int64_t)k * gsk]);
        b[s] = (colok && k4 + s < nk) ? v : 0.0;
      }
    }
  };
  // two groups of four K-steps (32 values of k) per trip, all operands
  // requested before the first product; K-step s of a group pairs slot q
  // with k = base + 4q + s
  for (int kb = klo; kb < khi; kb += 32) {
    double a0[4], b0[4], a1[4], b1[4];
    load_a(kb + 4 * q, a0);
    load_a(kb + 16 + 4 * q, a1);
    load_b(kb + 4 * q, b0);
    // past khi a1 is zero: any in-bounds, 4-aligned k serves
    load_b(min(kb + 16, (khi - 1) & ~3) + 4 * q, b1);
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b0[s], acc, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc, 0, 0, 0);
  }
  // D[i][j]: rows 16T + q + 4v, column col
  if (colok) {
    double *ub = U + o * ustride_o + col;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * T + q + 4 * v;
      if (r < R) ub[(int64_t)r * usk] = acc[v];
    }
  }
}

// S_r^a for all axes and orders r < p.  Workgroup: a 16 x 64 tile of
// (k1, k2) and a chunk [k0a, k0b) of k0; 64 x 4 threads, each owning 4 rows of
// the tile.  Each plane of P (tile plus p-1 halo rows and columns) is staged
// in LDS once for the axis-1 and axis-2 coefficients; every thread keeps its
// points' last p values along axis 0 in registers for the axis-0
// coefficients, which lag p-1 planes behind (the planes past the chunk are
// read as halo, those past the grid as zeros that no coefficient uses).
// The next two planes are in flight in registers while one is processed (two
// buffers, the plane loop unrolled by two and its count rounded up to even;
// unconditional in-bounds loads, zero fill where the values are used).  The
// axis-1 coefficient rows of the tile sit in LDS.
template <int PP>
__global__ void __launch_bounds__(256) k_deriv_scale_tiles(const double *__restrict__ P, int n0, int n1,
                                                           int n2, int K0C, DTab d0, DTab d1, DTab d2,
                                                           int act0, int act1, int act2,
                                                           unsigned long long *slots) {
  constexpr int TX = 64, TY = 16, RY = 4, H = PP - 1;
  constexpr int LYY = TY + H, LXX = TX + H;
  constexpr int NT = (LYY * LXX + 255) / 256;
  __shared__ double tile[LYY][LXX + 1];
  __shared__ double sd1[TY][PP][PP];   // axis-1 rows: sd1[k1 - k1a][r][q]
  // axis-0 rows of the chunk's planes, sd0[idx - k0a][r][q] (K0C <= 32),
  // staged once instead of loaded from global memory in every plane step
  __shared__ double sd0[32][PP][PP];
  const int tx = threadIdx.x & 63;
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k2a = blockIdx.x * TX, k1a = blockIdx.y * TY;
  const int k0a = blockIdx.z * K0C, k0b = min(n0, k0a + K0C);
  const int k2 = k2a + tx;
  const int64_t plane = (int64_t)n1 * n2;
  for (int e = threadIdx.x; e < TY * PP * PP; e += 256) {
    const int yl = e / (PP * PP), r = (e / PP) % PP, q = e % PP;
    const int k1 = k1a + yl;
    int rowoff = 0;
    for (int rr = 0; rr < r; ++rr) rowoff += n1 - rr;
    sd1[yl][r][q] = (act1 && q <= r && k1 <= n1 - 1 - r) ? d1.val[(int64_t)(rowoff + k1) * d1.L + q] : 0.0;
  }
  for (int e = threadIdx.x; e < K0C * PP * PP; e += 256) {
    const int il = e / (PP * PP), r = (e / PP) % PP, q = e % PP;
    const int idx = k0a + il;
    int rowoff = 0;
    for (int rr = 0; rr < r; ++rr) rowoff += n0 - rr;
    sd0[il][r][q] = (act0 && idx < k0b && q <= r && idx <= n0 - 1 - r)
                        ? d0.val[(int64_t)(rowoff + idx) * d0.L + q]
                        : 0.0;
  }
  // this thread's axis-2 coefficient rows (fixed k2)
  double dv2[PP][PP];
  {
    int rowoff = 0;
#pragma unroll
    for (int r = 0; r < PP; ++r) {
#pragma unroll
      for (int q = 0; q < PP; ++q)
        dv2[r][q] = (act2 && q <= r && k2 <= n2 - 1 - r) ? d2.val[(int64_t)(rowoff + k2) * d2.L + q] : 0.0;
      rowoff += n2 - r;
    }
  }
  // plane-invariant tile gathers: offsets within a plane and validity
  int toff[NT];
  unsigned tmask = 0;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int r = e / LXX, c = e - r * LXX;
    const int k1 = k1a + r, kk2 = k2a + c;
    const bool ok = e < LYY * LXX && k1 < n1 && kk2 < n2;
    toff[u] = ok ? k1 * n2 + kk2 : 0;
    tmask |= (unsigned)ok << u;
  }
  double win[RY][PP];
  double mx[3][PP];
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int q = 0; q < PP; ++q) win[j][q] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int r = 0; r < PP; ++r) mx[a][r] = 0.0;

  double bufA[NT], bufB[NT];
  bool inA = false, inB = false;
  auto gload = [&](double (&buf)[NT], bool &bin, int k0) {
    bin = k0 < n0;
    const double *base = P + (bin ? k0 : 0) * plane;
#pragma unroll
    for (int u = 0; u < NT; ++u) buf[u] = base[toff[u]];
  };
  auto step = [&](double (&buf)[NT], bool &bin, int k0) {
    // the plane whose axis-0 window completes here (uniform); its rows come
    // from sd0 (written before the first barrier below)
    const int idx = k0 - H;
    const bool do0 = act0 && idx >= k0a && idx < k0b;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e / LXX, c = e - r * LXX;
      if (e < LYY * LXX) tile[r][c] = (bin && ((tmask >> u) & 1)) ? buf[u] : 0.0;
    }
    __syncthreads();
    // past the chunk's last plane the prefetch re-reads that plane (cache hits,
    // never used) instead of the next chunk's planes
    gload(buf, bin, min(k0 + 2, k0b + H - 1));
    const bool own = k0 < k0b;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = ty + 4 * j, k1 = k1a + ly;
      const double c = tile[ly][tx];
#pragma unroll
      for (int q = 0; q + 1 < PP; ++q) win[j][q] = win[j][q + 1];
      win[j][PP - 1] = c;
      if (k1 >= n1 || k2 >= n2) continue;
      if (own && act2) {
#pragma unroll
        for (int r = 0; r < PP; ++r) {
          if (k2 <= n2 - 1 - r) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q <= r; ++q) sum += dv2[r][q] * tile[ly][tx + q];
            mx[2][r] = fmax(mx[2][r], fabs(sum));
          }
        }
      }
      if (own && act1) {
#pragma unroll
        for (int r = 0; r < PP; ++r) {
          if (k1 <= n1 - 1 - r) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q <= r; ++q) sum += sd1[ly][r][q] * tile[ly + q][tx];
            mx[1][r] = fmax(mx[1][r], fabs(sum));
          }
        }
      }
      if (do0) {
        const int il = idx - k0a;
#pragma unroll
        for (int r = 0; r < PP; ++r) {
          if (idx <= n0 - 1 - r) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q <= r; ++q) sum += sd0[il][r][q] * win[j][q];
            mx[0][r] = fmax(mx[0][r], fabs(sum));
          }
        }
      }
    }
  };
  const int npl = (k0b + H - k0a + 1) & ~1;
  gload(bufA, inA, k0a);
  // keep A's loads ahead of B's: the waits count loads in issue order
  asm volatile("" ::: "memory");
  gload(bufB, inB, k0a + 1);
  for (int k0 = k0a; k0 < k0a + npl; k0 += 2) {
    step(bufA, inA, k0);
    step(bufB, inB, k0 + 1);
  }
  // the workgroup's maxima: wavefront maxima through LDS, then one atomic
  // per (axis, order) on one slot copy (not one per wavefront)
  __shared__ double red[4][3 * PP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int r = 0; r < PP; ++r) {
      double v = mx[a][r];
      for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
      if (lane == 0) red[wv][a * PP + r] = v;
    }
  __syncthreads();
  const int act[3] = {act0, act1, act2};
  if (threadIdx.x < 3 * PP && act[threadIdx.x / PP]) {
    const int a = threadIdx.x / PP, r = threadIdx.x % PP;
    double m = red[0][threadIdx.x];
    for (int i = 1; i < 4; ++i) m = fmax(m, red[i][threadIdx.x]);
    const unsigned copy = (blockIdx.x * 7u + blockIdx.y * 131u + blockIdx.z * 1031u) % kSlotCopies;
    atomicMax(slots + (size_t)(kSlotS + a * kMaxP + r) * kSlotCopies + copy,
              (unsigned long long)__double_as_longlong(m));
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

DTab dtab(const Axis &X) { return DTab{X.D.len, X.D.col, X.D.val, X.D.L, X.n}; }
OmTab otab(const Axis &X) {
  return OmTab{X.Om.len, X.Om.col, X.Om.val, X.d_omT, X.Om.L, (int)X.m, X.n};
}

}  // namespace

template <int PP>
hipError_t deriv_scale_tiles(Handle &h) {
  const int n0 = h.ax[0].n, n1 = h.ax[1].n, n2 = h.ax[2].n;
  const unsigned gx = nblk(n2, 64), gy = nblk(n1, 16);
  int K0C = 32;
  while (K0C > 4 && (int64_t)gx * gy * nblk(n0, K0C) < 1024) K0C /= 2;
  const dim3 grid(gx, gy, nblk(n0, K0C));
  k_deriv_scale_tiles<PP><<<grid, 256, 0, h.stream>>>(h.P, n0, n1, n2, K0C, dtab(h.ax[0]), dtab(h.ax[1]),
                                                     dtab(h.ax[2]), h.ax[0].active, h.ax[1].active,
                                                     h.ax[2].active, h.slots);
  return hipGetLastError();
}

hipError_t launch_deriv_scale(Handle &h) {
  switch (h.p) {
    case 1: return deriv_scale_tiles<1>(h);
    case 2: return deriv_scale_tiles<2>(h);
    case 3: return deriv_scale_tiles<3>(h);
    case 4: return deriv_scale_tiles<4>(h);
    case 5: return deriv_scale_tiles<5>(h);
    case 6: return deriv_scale_tiles<6>(h);
    case 7: return deriv_scale_tiles<7>(h);
    case 8: return deriv_scale_tiles<8>(h);
    default: break;
  }
  const int n0 = h.ax[0].n, n1 = h.ax[1].n, n2 = h.ax[2].n;
  const int bs = n2 >= 256 ? 256 : ((n2 + 63) / 64) * 64;
  const int rows = 32;
  const dim3 grid(nblk(n2, bs), nblk(n1, rows), n0);
  k_deriv_scale<<<grid, bs, 0, h.stream>>>(h.P, n0, n1, n2, h.p, dtab(h.ax[0]), dtab(h.ax[1]),
                                           dtab(h.ax[2]), h.ax[0].active, h.ax[1].active,
                                           h.ax[2].active, rows, h.slots);
  return hipGetLastError();
}

template <typename TG>
hipError_t launch_jump_project(Handle &h, int a, const TG *g, double *U) {
  const Axis &X = h.ax[a];
  if (!getenv("MFA_VECTOR_JPROJ")) {
    // U = J_a applied along axis a on the matrix cores; U keeps the layout the
    // expansion reads (axis a replaced by the rows in place; for a = 2 the
    // rows outermost)
    const int R = (X.B - 1) * h.p;
    if (R == 0) return hipSuccess;
    const int64_t n0 = h.ax[0].n, n1 = h.ax[1].n, n2 = h.ax[2].n;
    int64_t ncol, go = 0, uo = 0, gsk, gsc, usk, outer = 1;
    if (a == 0) {
      ncol = n1 * n2; gsk = n1 * n2; gsc = 1; usk = n1 * n2;
    } else if (a == 1) {
      outer = n0; ncol = n2; go = n1 * n2; uo = (int64_t)R * n2; gsk = n2; gsc = 1; usk = n2;
    } else {
      ncol = n0 * n1; gsk = 1; gsc = n2; usk = n0 * n1;
    }
    const int nct = (int)((ncol + 15) / 16), nrt = (R + 15) / 16;
    const int64_t ntask = outer * nct * (int64_t)nrt;
    const unsigned grid = (unsigned)((ntask + 3) / 4);
    const int nk = X.n;
    if (a == 2)
      k_jproj_mfma<TG, true><<<grid, 256, 0, h.stream>>>(g, U, R, nrt, ncol, nct, go, uo, gsk, gsc, usk, nk,
                                                         ntask, X.J.col, X.J.len, X.J.val, X.J.L);
    else
      k_jproj_mfma<TG, false><<<grid, 256, 0, h.stream>>>(g, U, R, nrt, ncol, nct, go, uo, gsk, gsc, usk, nk,
                                                          ntask, X.J.col, X.J.len, X.J.val, X.J.L);
    return hipGetLastError();
  }
  const size_t jbytes = sizeof(double) * (size_t)(X.B - 1) * h.p * X.J.L;
  if (a == 2 && (int64_t)X.n * 8 <= 32768 && jbytes <= 16384) {
    const int64_t nlines = (int64_t)h.ax[0].n * h.ax[1].n;
    // staged lines: float for a float or BF16 residual (exact), else double;
    // up to 32 KB of them per workgroup
    using SG = typename std::conditional<sizeof(TG) <= 4, float, double>::type;
    const int ldg = X.n | 1;
    const int LPB = std::max(1, std::min(64, 32768 / ((int)sizeof(SG) * ldg)));
    k_jump_project_lines<TG, SG><<<nblk(nlines, LPB), 256, sizeof(SG) * LPB * ldg + jbytes, h.stream>>>(
        g, U, nlines, X.n, X.B - 1, h.p, LPB, X.J.col, X.J.len, X.J.val, X.J.L);
    return hipGetLastError();
  }
  if (a == 2) {
    const int64_t nlines = (int64_t)h.ax[0].n * h.ax[1].n;
    const dim3 grid(nblk(nlines, 256), X.B - 1);
    k_jump_project_inner<TG><<<grid, 256, 0, h.stream>>>(g, U, nlines, h.ax[2].n, X.B - 1, h.p,
                                                         X.J.col, X.J.len, X.J.val, X.J.L);
    return hipGetLastError();
  }
  int d[3] = {h.ax[0].n, h.ax[1].n, h.ax[2].n};
  d[a] = X.B - 1;
  const int bs = d[2] >= 256 ? 256 : ((d[2] + 63) / 64) * 64;
  const dim3 grid(nblk(d[2], bs), d[1], d[0]);
  k_jump_project<TG><<<grid, bs, sizeof(double) * h.p * X.J.L, h.stream>>>(g, U, a, h.ax[0].n, h.ax[1].n,
                                                                            h.ax[2].n, X.B - 1,
                                                h.p, X.J.col, X.J.len, X.J.val, X.J.L);
  return hipGetLastError();
}
template hipError_t launch_jump_project<double>(Handle &, int, const double *, double *);
template hipError_t launch_jump_project<float>(Handle &, int, const float *, double *);
template hipError_t launch_jump_project<__hip_bfloat16>(Handle &, int, const __hip_bfloat16 *, double *);

// U = J_a applied along axis a of the residual (dims with axis a of length R).
hipError_t launch_jump_expand(Handle &h, int a, const double *U) {
  const Axis &X = h.ax[a];
  const int R = (X.B - 1) * h.p;
  int64_t d[3] = {h.ax[0].n, h.ax[1].n, h.ax[2].n};
  d[a] = R;
  // U has axis a replaced by the R interface rows in place, except for the
  // contiguous axis (a = 2), whose projection stores the rows outermost
  int64_t st[3] = {d[1] * d[2], d[2], 1};
  if (a == 2) {
    st[2] = d[0] * d[1];
    st[0] = d[1];
    st[1] = 1;
  }
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
  // data points per workgroup: 8 (of 4, 8, 16 the fastest on a 256 x 256 x
  // 192 grid: more workgroups, all resident at once), fewer for long rows
  const int jb = nc <= 768 ? 8 : (nc <= 1536 ? 4 : 1);
  const unsigned grid = (unsigned)((int64_t)R * ((Ob.m + jb - 1) / jb));
  // widest union of the Om_b column ranges (owners' free sets) over a group
  // of jb consecutive data points
  int wmax = 1;
  for (int64_t i0 = 0; i0 < Xb.m; i0 += jb) {
    int lo = 1 << 30, hi = 0;
    for (int64_t i = i0; i < std::min<int64_t>(Xb.m, i0 + jb); ++i) {
      const Block &B = Xb.blk[Xb.pown[i]];
      lo = std::min(lo, B.F0);
      hi = std::max(hi, B.F1);
    }
    wmax = std::max(wmax, hi - lo);
  }
  const size_t lds = sizeof(double) * jb * (nc + wmax) + sizeof(int) * 2 * jb;
  if (lds > 64 * 1024) return hipErrorInvalidValue;
#define MFA_JE(JB)                                                                                  \
  k_jump_expand<JB><<<grid, 256, lds, h.stream>>>(U, R, st[a], st[oth[0]], sc, Ob, Oc, has_c, h.p, \
                                                 kSlotJ + a * kMaxP, h.slots, wmax)
  if (jb == 8) MFA_JE(8);
  else if (jb == 4) MFA_JE(4);
  else MFA_JE(1);
#undef MFA_JE
  return hipGetLastError();
}

}  // namespace mfa
