// Streaming passes between the data grid and the control grid (Section 2.1:
// the tensor-product basis N = N_0 x N_1 x N_2 of eq. nurbs-basis, W = 1):
//
//   projection  c = (N_0^T x N_1^T x N_2^T) Q      (the right-hand side N^T Q)
//   decode      f = (N_0 x N_1 x N_2) P            (any derivative order per axis)
//
// Each is two kernels.  The inner kernel handles axes 1 and 2 of one slab i0
// (axis 2 contiguous, staged through LDS); the outer kernel handles axis 0
// with one thread per contiguous column.  Every element of the data grid is
// read (projection) or written (decode) once, up to the few rows that two
// neighbouring chunks share.
//
// Along an axis with m data points and n control points, point i touches the
// p+1 control points span(i)-p .. span(i), and span grows by at most one from
// one point to the next (m >= n).  A pass that walks the points in order
// therefore keeps just p+1 open control rows in registers: when the span
// moves on, the oldest row has received all its contributions and is written
// (projection), or the next control row is read (decode).
#include <cstdlib>

#include "mfa_internal.hpp"

namespace mfa {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

__device__ __forceinline__ int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }


// span(i) = min(n-1, p + floor(i (n-p) / (m-1))): the first point whose span
// is >= s, and the last point whose span is <= s.
__device__ __forceinline__ int64_t first_span_ge(int s, int64_t m, int n, int p) {
  if (s <= p) return 0;
  return cdiv((int64_t)(s - p) * (m - 1), n - p);
}
__device__ __forceinline__ int64_t last_span_le(int s, int64_t m, int n, int p) {
  if (s >= n - 1) return m - 1;
  return cdiv((int64_t)(s - p + 1) * (m - 1), n - p) - 1;
}

// Basis rows of one axis: point i has the p+1 values val[i*L + q] at control
// points span[i]-p+q.
struct Rows {
  const int *span;
  const double *val;
  int L;
  int64_t m;
  int n;
};

// ---------------------------------------------------------------------------
// projection, inner: out[i0][k1][k2] = sum_{i1,i2} N_1[i1][k1] N_2[i2][k2] Q[i0][i1][i2]
// Workgroup: slab i0 (grid.y), a chunk [K1a, K1b) of k1 and a chunk of
// blockDim k2 (grid.x).  RI rows of Q (the columns the k2 chunk needs) are
// staged in LDS; each thread contracts them along axis 2 for its k2 with its
// N_2^T row held in registers (NTR values at most), then folds the result
// into the p+1 open k1 rows.
template <typename TQ, int P, int RI, int NTR, int NCW>
__global__ void __launch_bounds__(256) k_proj_inner(const TQ *__restrict__ Q, double *__restrict__ out,
                                                    int64_t m1, int64_t m2, int n1, int n2, int K1C,
                                                    Rows r1, const int *__restrict__ nt2col,
                                                    const int *__restrict__ nt2len,
                                                    const double *__restrict__ nt2val, int LT2,
                                                    int maxrows) {
  extern __shared__ __align__(16) unsigned char smem[];
  // LDS: this chunk's axis-1 weights and spans, then the staged rows of Q
  double *sw = reinterpret_cast<double *>(smem);
  int *ss = reinterpret_cast<int *>(sw + (size_t)maxrows * (P + 1));
  TQ *rows = reinterpret_cast<TQ *>(ss + ((maxrows + 3) & ~3));
  const int BS = blockDim.x, tid = threadIdx.x;
  const int nk1c = (n1 + K1C - 1) / K1C;
  const int ck1 = blockIdx.x % nk1c, ck2 = blockIdx.x / nk1c;
  const int64_t i0 = blockIdx.y;
  const int K1a = ck1 * K1C, K1b = min(n1, K1a + K1C);
  const int K2a = ck2 * BS, K2b = min(n2, K2a + BS);
  const int k2 = K2a + tid;
  const bool act = k2 < K2b;
  const int64_t c_lo = first_span_ge(max(K2a, P), m2, n2, P);
  const int64_t c_hi = last_span_le(min(K2b - 1 + P, n2 - 1), m2, n2, P) + 1;
  const int W = (int)(c_hi - c_lo);
  const int64_t r_lo = first_span_ge(max(K1a, P), m1, n1, P);
  const int64_t r_hi = last_span_le(min(K1b - 1 + P, n1 - 1), m1, n1, P) + 1;

  // this thread's row of N_2^T: contiguous data points from col0
  double tv[NTR];
  int len = 0, off = 0;
  if (act) {
    len = nt2len[k2];
    off = (int)(nt2col[(int64_t)k2 * LT2] - c_lo);
  }
#pragma unroll
  for (int t = 0; t < NTR; ++t) tv[t] = (act && t < len) ? nt2val[(int64_t)k2 * LT2 + t] : 0.0;

  const int nrow = (int)(r_hi - r_lo);
  for (int e = tid; e < nrow * (P + 1); e += BS) {
    const int rr = e / (P + 1);
    sw[e] = r1.val[(r_lo + rr) * r1.L + (e - rr * (P + 1))];
  }
  for (int e = tid; e < nrow; e += BS) ss[e] = r1.span[r_lo + e];
  __syncthreads();
  double acc[P + 1];
#pragma unroll
  for (int q = 0; q <= P; ++q) acc[q] = 0.0;
  int cur = ss[0];
  double *dst = out + (i0 * n1) * (int64_t)n2 + k2;

  // The next group of RI rows (W <= NCW * BS columns) is loaded into
  // registers while the current one is contracted; the loads use clamped
  // in-bounds indices and carry no branches (rows past the group and columns
  // past W are never stored or read).
  // NTR zeros after the last staged row (the row stores never reach them)
  for (int e = tid; e < NTR; e += BS) rows[RI * W + e] = (TQ)0;
  TQ pre[RI][NCW];
  auto fetch = [&](int64_t g) {
    const int nr = (int)min((int64_t)RI, r_hi - g);
    const TQ *src = Q + (i0 * m1 + g) * m2 + c_lo;
#pragma unroll
    for (int rr = 0; rr < RI; ++rr)
#pragma unroll
      for (int cw = 0; cw < NCW; ++cw)
        pre[rr][cw] = src[(int64_t)min(rr, nr - 1) * m2 + min(tid + cw * BS, W - 1)];
  };
  fetch(r_lo);
  for (int64_t g = r_lo; g < r_hi; g += RI) {
    const int nr = (int)min((int64_t)RI, r_hi - g);
    __syncthreads();   // the previous group's rows have been consumed
#pragma unroll
    for (int rr = 0; rr < RI; ++rr)
#pragma unroll
      for (int cw = 0; cw < NCW; ++cw)
        if (rr < nr && tid + cw * BS < W) rows[rr * W + tid + cw * BS] = pre[rr][cw];
    __syncthreads();
    fetch(min(g + RI, r_hi - 1));
    // axis 2 for RB rows at a time as independent chains (rows past nr are
    // stale and never used; RI is a multiple of RB).  Taps past len have
    // zero weights and read the next values of the staged rows, or the
    // zeroed pad after the last row, so every term is exact and in bounds.
    constexpr int RB = NTR <= 12 ? 4 : (NTR <= 24 ? 2 : 1);
    static_assert(RI % RB == 0, "row batches tile the group");
    for (int r0 = 0; r0 < nr; r0 += RB) {
      double vb[RB];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const TQ *row = rows + (r0 + b) * W + off;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < NTR; ++t) v += tv[t] * (double)row[t];
        vb[b] = v;
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (r0 + b >= nr) break;
        const int64_t i1 = g + r0 + b;
        const double v = vb[b];
        const int s = ss[i1 - r_lo];
        if (s != cur) {   // s == cur + 1: row cur-p is complete
          const int k1 = cur - P;
          if (act && k1 >= K1a && k1 < K1b) dst[(int64_t)k1 * n2] = acc[0];
#pragma unroll
          for (int q = 0; q < P; ++q) acc[q] = acc[q + 1];
          acc[P] = 0.0;
          cur = s;
        }
        const double *w = sw + (i1 - r_lo) * (P + 1);
#pragma unroll
        for (int q = 0; q <= P; ++q) acc[q] += w[q] * v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    const int k1 = cur - P + q;
    if (act && k1 >= K1a && k1 < K1b) dst[(int64_t)k1 * n2] = acc[q];
  }
}

// ---------------------------------------------------------------------------
// projection, outer: out[k0][j] = sum_i0 N_0[i0][k0] in[i0][j] for a chunk
// [K0a, K0b) of k0 (grid.y) and 256 consecutive columns j (grid.x).
template <int P>
__global__ void __launch_bounds__(256) k_proj_outer(const double *__restrict__ in, double *__restrict__ out,
                                                    int64_t J, int n0, int K0C, Rows r0, int maxrows) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *sw = reinterpret_cast<double *>(smem);
  int *ss = reinterpret_cast<int *>(sw + (size_t)maxrows * (P + 1));
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < J;
  const int K0a = blockIdx.y * K0C, K0b = min(n0, K0a + K0C);
  const int64_t r_lo = first_span_ge(max(K0a, P), r0.m, n0, P);
  const int64_t r_hi = last_span_le(min(K0b - 1 + P, n0 - 1), r0.m, n0, P) + 1;
  const int nrow = (int)(r_hi - r_lo);
  for (int e = threadIdx.x; e < nrow * (P + 1); e += blockDim.x) {
    const int rr = e / (P + 1);
    sw[e] = r0.val[(r_lo + rr) * r0.L + (e - rr * (P + 1))];
  }
  for (int e = threadIdx.x; e < nrow; e += blockDim.x) ss[e] = r0.span[r_lo + e];
  __syncthreads();
  double acc[P + 1];
#pragma unroll
  for (int q = 0; q <= P; ++q) acc[q] = 0.0;
  int cur = ss[0];
  const double *src = in + (act ? j : 0);
  constexpr int U = 4;
  for (int64_t g = r_lo; g < r_hi; g += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (act && g + u < r_hi) ? src[(g + u) * J] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i0 = g + u;
      if (i0 < r_hi) {
        const int s = ss[i0 - r_lo];
        if (s != cur) {
          const int k0 = cur - P;
          if (act && k0 >= K0a && k0 < K0b) out[(int64_t)k0 * J + j] = acc[0];
#pragma unroll
          for (int q = 0; q < P; ++q) acc[q] = acc[q + 1];
          acc[P] = 0.0;
          cur = s;
        }
        const double *w = sw + (i0 - r_lo) * (P + 1);
#pragma unroll
        for (int q = 0; q <= P; ++q) acc[q] += w[q] * v[u];
      }
    }
  }
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    const int k0 = cur - P + q;
    if (act && k0 >= K0a && k0 < K0b) out[(int64_t)k0 * J + j] = acc[q];
  }
}

// ---------------------------------------------------------------------------
// decode, outer: out[i0][j] = sum_q N_0[i0][q] in[span0(i0)-p+q][j] for a
// chunk of data rows i0 (grid.y) and 256 consecutive columns j (grid.x).  The
// p+1 control rows under the current span sit in registers, the next one is
// read ahead.
template <int P, typename TO>
__global__ void __launch_bounds__(256) k_dec_outer(const double *__restrict__ in, TO *__restrict__ out,
                                                   int64_t J, int I0C, Rows r0) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *sw = reinterpret_cast<double *>(smem);                // [I0C][P+1]
  int *ss = reinterpret_cast<int *>(sw + (size_t)I0C * (P + 1));  // [I0C]
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < J;
  const int64_t I0a = (int64_t)blockIdx.y * I0C, I0b = min(r0.m, I0a + I0C);
  const int nrow = (int)(I0b - I0a);
  for (int e = threadIdx.x; e < nrow * (P + 1); e += blockDim.x) {
    const int rr = e / (P + 1);
    sw[e] = r0.val[(I0a + rr) * r0.L + (e - rr * (P + 1))];
  }
  for (int e = threadIdx.x; e < nrow; e += blockDim.x) ss[e] = r0.span[I0a + e];
  __syncthreads();
  if (!act) return;
  int cur = ss[0];
  double win[P + 1];
#pragma unroll
  for (int q = 0; q <= P; ++q) win[q] = in[(int64_t)(cur - P + q) * J + j];
  double nxt = cur + 1 < r0.n ? in[(int64_t)(cur + 1) * J + j] : 0.0;
  for (int rr = 0; rr < nrow; ++rr) {
    const int s = ss[rr];
    if (s != cur) {   // s == cur + 1
#pragma unroll
      for (int q = 0; q < P; ++q) win[q] = win[q + 1];
      win[P] = nxt;
      cur = s;
      nxt = cur + 1 < r0.n ? in[(int64_t)(cur + 1) * J + j] : 0.0;
    }
    const double *w = sw + rr * (P + 1);
    double v = 0.0;
#pragma unroll
    for (int q = 0; q <= P; ++q) v += w[q] * win[q];
    out[(I0a + rr) * J + j] = (TO)v;
  }
}

// Residual reduction slots: kSlotCopies copies of max |d| (non-negative
// double bit patterns, atomic max) followed by kSlotCopies copies of the sum
// of d^2 (doubles, atomic add).
__device__ __forceinline__ void res_reduce(unsigned long long *rs, double mx, double sq) {
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    sq += __shfl_xor(sq, off, 64);
  }
  if (__lane_id() == 0) {
    const unsigned copy = (blockIdx.x * 7u + blockIdx.y * 131u + (threadIdx.x >> 6)) % kSlotCopies;
    atomicMax(rs + copy, (unsigned long long)__double_as_longlong(mx));
    atomicAdd(reinterpret_cast<double *>(rs + kSlotCopies + copy), sq);
  }
}

// ---------------------------------------------------------------------------
// decode, inner: out[i0][i1][i2] = sum_{q1,q2} N_1[i1][q1] N_2[i2][q2]
//                                  in[i0][span1(i1)-p+q1][span2(i2)-p+q2]
// Workgroup: slab i0 (grid.y) and a chunk of data rows i1 (grid.x).  Phase A:
// thread k2 (< n2 <= blockDim) expands axis 1 from its p+1 open control rows
// (registers) into RI rows in LDS.  Phase B: thread i2 (IS points per thread,
// their N_2 rows in registers) expands axis 2 from LDS and writes the output.
// RES: `out` holds the data Q instead (read only); each decoded value d is
// compared with it and max |Q - d| and sum (Q - d)^2 go to `rs`.
template <typename TO, int P, int RI, int IS, bool RES>
__global__ void __launch_bounds__(256) k_dec_inner(const double *__restrict__ in, TO *__restrict__ out,
                                                   int64_t m1, int64_t m2, int n1, int n2, int I1C,
                                                   Rows r1, Rows r2, unsigned long long *rs) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *rows = reinterpret_cast<double *>(smem);                // [RI][n2]
  double *sw = rows + (size_t)RI * n2;                            // [I1C][P+1] axis-1 weights
  int *ss = reinterpret_cast<int *>(sw + (size_t)I1C * (P + 1));  // [I1C] axis-1 spans
  const int BS = blockDim.x, tid = threadIdx.x;
  const int64_t i0 = blockIdx.y;
  const int64_t I1a = (int64_t)blockIdx.x * I1C, I1b = min(m1, I1a + I1C);
  {
    const int nrow = (int)(I1b - I1a);
    for (int e = tid; e < nrow * (P + 1); e += BS) {
      const int rr = e / (P + 1);
      sw[e] = r1.val[(I1a + rr) * r1.L + (e - rr * (P + 1))];
    }
    for (int e = tid; e < nrow; e += BS) ss[e] = r1.span[I1a + e];
  }
  __syncthreads();
  const bool actk = tid < n2;
  const double *slab = in + i0 * (int64_t)n1 * n2 + (actk ? tid : 0);

  // phase-B rows of N_2 for this thread's points
  double w2[IS][P + 1];
  int c2[IS];
#pragma unroll
  for (int s = 0; s < IS; ++s) {
    const int64_t i2 = tid + (int64_t)s * BS;
    const bool ok = i2 < m2;
    c2[s] = ok ? r2.span[i2] - P : 0;
#pragma unroll
    for (int q = 0; q <= P; ++q) w2[s][q] = ok ? r2.val[i2 * r2.L + q] : 0.0;
  }

  int cur = ss[0];
  double win[P + 1];
#pragma unroll
  for (int q = 0; q <= P; ++q) win[q] = slab[(int64_t)(cur - P + q) * n2];
  TO *dst = out + i0 * m1 * m2;
  double rmax = 0.0, rsq = 0.0;

  for (int64_t g = I1a; g < I1b; g += RI) {
    const int nr = (int)min((int64_t)RI, I1b - g);
    // the group's rows advance the span adv <= nr <= RI times: control rows
    // cur+1 .. cur+adv of this column are requested together, one wait per
    // group (the remaining registers re-read the last of them, a cache hit)
    const int adv = ss[g + nr - 1 - I1a] - cur;
    double nx[RI];
#pragma unroll
    for (int u = 0; u < RI; ++u) nx[u] = slab[(int64_t)(cur + min(u + 1, adv)) * n2];
    for (int rr = 0; rr < nr; ++rr) {
      const int64_t i1 = g + rr;
      const int s = ss[i1 - I1a];
      if (s != cur) {
#pragma unroll
        for (int q = 0; q < P; ++q) win[q] = win[q + 1];
        win[P] = nx[0];
#pragma unroll
        for (int u = 0; u + 1 < RI; ++u) nx[u] = nx[u + 1];
        cur = s;
      }
      const double *w = sw + (i1 - I1a) * (P + 1);
      double v = 0.0;
#pragma unroll
      for (int q = 0; q <= P; ++q) v += w[q] * win[q];
      if (actk) rows[rr * n2 + tid] = v;
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double *row = rows + rr * n2;
      TO *o = dst + (g + rr) * m2;
#pragma unroll
      for (int s = 0; s < IS; ++s) {
        const int64_t i2 = tid + (int64_t)s * BS;
        if (i2 < m2) {
          double v = 0.0;
#pragma unroll
          for (int q = 0; q <= P; ++q) v += w2[s][q] * row[c2[s] + q];
          if (RES) {
            const double d = (double)o[i2] - v;
            rmax = fmax(rmax, fabs(d));
            rsq += d * d;
          } else {
            o[i2] = (TO)v;
          }
        }
      }
    }
    __syncthreads();   // rows are rewritten by the next group
  }
  if (RES) res_reduce(rs, rmax, rsq);
}

// ---------------------------------------------------------------------------
// decode, axes 1 and 2 on the matrix cores (FP32 output).
//
// For one slab i0 and a tile of 16 data rows i1 = 16 I + j the slab's part
// of the output is two banded products, U = N_1[tile] T (T the slab after
// axis 0) and out = U N_2^T, each blocked into dense 16 x 16 tiles and run
// as v_mfma_f32_16x16x4_f32 (FP32 operands, FP32 accumulation).  Operand
// layout of that instruction (one wave): A[i][k] in lane i + 16 k, B[k][j]
// in lane j + 16 k, D[i][j] in lane j + 16 (i / 4), register i % 4.
//
// Step 1 forms U transposed, one tile of 16 control columns k2 at a time:
// D[k2][i1] = sum_k1 T[k1][k2] N_1[i1][k1] over the window of 4 KS control
// rows k1 that starts at klo1(I), so that a lane ends up holding
// U[16 I + lane % 16][16 J + 4 (lane / 16) + v] in register v.
// Step 2 forms an output tile of 16 points i2, transposed:
// D[i2][i1] = sum_k2 N_2[i2][k2] U[i1][k2].  The 16 columns of a U tile
// enter as four K-steps v, step v pairing k2 = 16 J + 4 k + v with operand
// slot k; the B operand of step v is then a lane's own U register v (no
// data movement between the two products) and the A operand comes from a
// table of N_2 laid out the same way, staged in LDS once per workgroup.  A
// lane ends up holding out[16 I + lane % 16][16 J2 + 4 (lane / 16) + w],
// w = 0..3: one 16-byte store.  The control window of an output tile starts
// in U tile J0(J2) and reaches at most into J0 + 1 (checked on the host).
// The loop runs over U tiles J and, inside, over the output tiles with
// J0 = J; U tiles J and J + 1 sit in registers, the T operands of J + 2 and
// J + 3 are in flight.  Vector memory then carries only those T requests and
// the stores, so that waiting for one U tile's operands never waits for a
// later request (the counters are in order).  Each wave owns one (i0, I).

// Operand tables, built per decode from the basis rows of the requested
// derivative orders:
//   w1t[I][lane][s]      N_1[16 I + lane % 16][klo1(I) + 4 s + lane / 16]
//   klo1[I]              span_1(16 I) - p
//   w2t[J2][jj][lane][v] N_2[16 J2 + lane % 16][16 (J0 + jj) + 4 (lane / 16) + v]
//   j0n[J2]              2 J0 + (window reaches tile J0 + 1), J0 = (span_2(16 J2) - p) / 16
//   j2beg[J]             first output tile J2 with J0(J2) >= J, J = 0..ntk
// (zero outside a row's p+1 non-zeros and past the last data point).
template <int P>
__global__ void __launch_bounds__(256) k_dec_tab(Rows r1, Rows r2, int nt1, int nt2, int ntk,
                                                 float *__restrict__ w1t, int *__restrict__ klo1,
                                                 float *__restrict__ w2t, int *__restrict__ j0n,
                                                 int *__restrict__ j2beg) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n1e = (int64_t)nt1 * 64, n2e = (int64_t)nt2 * 128;
  auto j0_of = [&](int J2) { return (r2.span[16 * (int64_t)J2] - P) / 16; };
  if (t < n1e) {
    const int I = (int)(t >> 6), l = (int)(t & 63);
    const int64_t i1 = 16 * (int64_t)I + (l & 15);
    const int lo = r1.span[16 * (int64_t)I] - P;
    if (l == 0) klo1[I] = lo;
    const bool ok = i1 < r1.m;
    const int first = ok ? r1.span[i1] - P : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = lo + 4 * s + (l >> 4) - first;
      w1t[t * 4 + s] = ok && q >= 0 && q <= P ? (float)r1.val[i1 * r1.L + q] : 0.0f;
    }
  } else if (t < n1e + n2e) {
    const int64_t u = t - n1e;
    const int J2 = (int)(u >> 7), jj = (int)((u >> 6) & 1), l = (int)(u & 63);
    const int64_t i2 = 16 * (int64_t)J2 + (l & 15);
    const int J0 = j0_of(J2);
    if (jj == 0 && l == 0) {
      const int64_t last = min(16 * (int64_t)J2 + 15, r2.m - 1);
      j0n[J2] = 2 * J0 + (r2.span[last] / 16 > J0 ? 1 : 0);
    }
    const bool ok = i2 < r2.m;
    const int first = ok ? r2.span[i2] - P : 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * (J0 + jj) + 4 * (l >> 4) + v - first;
      w2t[u * 4 + v] = ok && q >= 0 && q <= P ? (float)r2.val[i2 * r2.L + q] : 0.0f;
    }
  } else if (t <= n1e + n2e + ntk) {
    const int J = (int)(t - n1e - n2e);
    int J2 = 0;
    while (J2 < nt2 && j0_of(J2) < J) ++J2;
    j2beg[J] = J2;
  }
}

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 d) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
}

template <typename TI, bool V4, int NTK>
__global__ void __launch_bounds__(512) k_dec_mfma(const TI *__restrict__ T, float *__restrict__ out, int64_t m1,
                                                  int64_t m2, int n1, int n2, int nt1, int nt2,
                                                  const float *__restrict__ w1t, const int *__restrict__ klo1,
                                                  const float *__restrict__ w2t, const int *__restrict__ j0n,
                                                  const int *__restrict__ j2beg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ntk = (n2 + 15) >> 4;   // <= NTK
  floatx4 *sw2 = reinterpret_cast<floatx4 *>(smem);   // [nt2][2][64]
  int *sfl = reinterpret_cast<int *>(sw2 + (size_t)nt2 * 128);   // [nt2] two-tile flags
  int *sbeg = sfl + nt2;                                          // [ntk + 1]
  {
    const floatx4 *src = reinterpret_cast<const floatx4 *>(w2t);
    for (int e = threadIdx.x; e < nt2 * 128; e += blockDim.x) sw2[e] = src[e];
    for (int e = threadIdx.x; e < nt2; e += blockDim.x) sfl[e] = j0n[e] & 1;
    for (int e = threadIdx.x; e <= ntk; e += blockDim.x) sbeg[e] = j2beg[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int I = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (I >= nt1) return;   // whole waves, after the only barrier
  const int g = lane >> 4, c = lane & 15;
  const TI *Ts = T + (int64_t)blockIdx.y * n1 * n2;
  const floatx4 b1 = *reinterpret_cast<const floatx4 *>(w1t + ((int64_t)I * 64 + lane) * 4);
  const int lo1 = klo1[I];
  int roff[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) roff[s] = min(lo1 + 4 * s + g, n1 - 1) * n2;
  // Every T operand of the wave is requested at once (tile indices past the
  // last are clamped to it: in bounds, never read by an output tile), then
  // the U tiles are formed in order.
  float tv[NTK][4];
#pragma unroll
  for (int J = 0; J < NTK; ++J) {
    const int col = min(16 * min(J, ntk - 1) + c, n2 - 1);
#pragma unroll
    for (int s = 0; s < 4; ++s) tv[J][s] = (float)Ts[roff[s] + col];
  }
  floatx4 U[NTK];
#pragma unroll
  for (int J = 0; J < NTK; ++J) {
    floatx4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) d = mfma_f32(tv[J][s], b1[s], d);
    U[J] = d;
  }
  const int64_t i1 = 16 * (int64_t)I + c;
  const bool rowok = i1 < m1;
  float *oslab = out + (int64_t)blockIdx.y * m1 * m2;
  float *orow = oslab + min(i1, m1 - 1) * m2 + 4 * g;
  const floatx4 *a2 = sw2 + lane;
  // Output tiles go out in pairs (J2 even, J2 + 1): the pair's 16 rows x 32
  // columns are regrouped across lanes so that each store instruction covers
  // 8 whole rows of 128 bytes (a lane takes 4 columns of one row from the
  // lane that formed them), instead of 16 rows of 64 bytes per tile.
  auto store_pair = [&](const floatx4 &d0, const floatx4 &d1, int J2a) {
    const int q = lane & 7;   // column block of 4 within the pair
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int sc = 8 * k + (lane >> 3);           // row within the tile
      const int addr = (((q & 3) << 4) + sc) << 2;  // lane holding that row's block q
      floatx4 v;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const float x0 = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(d0[w])));
        const float x1 = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(d1[w])));
        v[w] = q < 4 ? x0 : x1;
      }
      const int64_t r = 16 * (int64_t)I + sc, col = 16 * (int64_t)J2a + 4 * q;
      if (r < m1 && col < m2) *reinterpret_cast<floatx4 *>(oslab + r * m2 + col) = v;
    }
  };
  floatx4 dprev = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int J = 0; J < NTK; ++J) {
    const floatx4 ua = U[J], ub = U[J + 1 < NTK ? J + 1 : J];
    // output tiles whose control window starts in U tile J (none past ntk)
    const int e0 = J < ntk ? __builtin_amdgcn_readfirstlane(sbeg[J]) : 0;
    const int e1 = J < ntk ? __builtin_amdgcn_readfirstlane(sbeg[J + 1]) : 0;
    for (int J2 = e0; J2 < e1; ++J2) {
      const floatx4 a0 = a2[J2 * 128];
      const int two = __builtin_amdgcn_readfirstlane(sfl[J2]);
      floatx4 d = {0.f, 0.f, 0.f, 0.f};
      d = mfma_f32(a0[0], ua[0], d);
      d = mfma_f32(a0[1], ua[1], d);
      d = mfma_f32(a0[2], ua[2], d);
      d = mfma_f32(a0[3], ua[3], d);
      if (two) {
        const floatx4 a1 = a2[J2 * 128 + 64];
        d = mfma_f32(a1[0], ub[0], d);
        d = mfma_f32(a1[1], ub[1], d);
        d = mfma_f32(a1[2], ub[2], d);
        d = mfma_f32(a1[3], ub[3], d);
      }
      const int64_t i2 = 16 * (int64_t)J2;
      if (V4) {
        if (J2 & 1) {
          store_pair(dprev, d, J2 - 1);
        } else if (J2 + 1 < nt2) {
          dprev = d;
        } else if (rowok && i2 + 4 * g < m2) {
          *reinterpret_cast<floatx4 *>(orow + i2) = d;
        }
      } else if (rowok) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
          if (i2 + 4 * g + w < m2) orow[i2 + w] = d[w];
      }
    }
  }
}

inline unsigned nblk(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

Rows rows_of(const Axis &X, int r) {
  return Rows{X.d_span, X.N[r].val, X.N[r].L, X.m, X.n};
}

constexpr int kProjRI = 8;
constexpr int kProjPad = 48;   // the largest N_2^T row length the projection takes
constexpr int kDecRI = 8;

int pick_chunk(int64_t parallel, int n, int lo) {
  // largest chunk in {64, 32, 16, lo} that still gives >= 2048 workgroups
  for (int c : {64, 32, 16})
    if (c >= lo && parallel * ((n + c - 1) / c) >= 2048) return c;
  return lo;
}

template <int P>
hipError_t project_p(Handle &h, const void *q, bool f32) {
  const Axis &X0 = h.ax[0], &X1 = h.ax[1], &X2 = h.ax[2];
  const int64_t m0 = X0.m, m1 = X1.m, m2 = X2.m;
  const int n0 = X0.n, n1 = X1.n, n2 = X2.n;
  // k2 chunk: up to 256 threads, narrower when the grid would be too small
  int BS = n2 >= 256 ? 256 : ((n2 + 63) / 64) * 64;
  while (BS > 64 && m0 * nblk(n1, 8) * nblk(n2, BS) < 1024) BS = ((BS / 2 + 63) / 64) * 64;
  const int nk2c = (n2 + BS - 1) / BS;
  const int K1C = pick_chunk(m0 * nk2c, n1, 8);
  const int nk1c = (n1 + K1C - 1) / K1C;
  // widest column range one k2 chunk needs (host copy of the span rule)
  auto first_ge = [&](int s) -> int64_t {
    return s <= P ? 0 : ((int64_t)(s - P) * (m2 - 1) + (n2 - P) - 1) / (n2 - P);
  };
  auto last_le = [&](int s) -> int64_t {
    return s >= n2 - 1 ? m2 - 1 : ((int64_t)(s - P + 1) * (m2 - 1) + (n2 - P) - 1) / (n2 - P) - 1;
  };
  int64_t W = 0;
  for (int c = 0; c < nk2c; ++c) {
    const int a = c * BS, b = std::min(n2, a + BS);
    W = std::max(W, last_le(std::min(b - 1 + P, n2 - 1)) + 1 - first_ge(std::max(a, P)));
  }
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  // most axis-1 rows one k1 chunk touches (same rule as the kernel)
  auto rows_of_chunk = [&](int64_t m, int n, int a, int b) -> int64_t {
    const int s0 = std::max(a, P), s1 = std::min(b - 1 + P, n - 1);
    const int64_t lo = s0 <= P ? 0 : ((int64_t)(s0 - P) * (m - 1) + (n - P) - 1) / (n - P);
    const int64_t hi = s1 >= n - 1 ? m - 1 : ((int64_t)(s1 - P + 1) * (m - 1) + (n - P) - 1) / (n - P) - 1;
    return hi + 1 - lo;
  };
  int maxrows1 = 0;
  for (int c = 0; c < nk1c; ++c)
    maxrows1 = (int)std::max<int64_t>(maxrows1, rows_of_chunk(m1, n1, c * K1C, std::min(n1, c * K1C + K1C)));
  // staged rows plus a pad of the largest N_2^T row length (zeros the
  // kernel's contraction may read past the last row)
  const size_t lds = (size_t)maxrows1 * (P + 1) * sizeof(double) + ((maxrows1 + 3) & ~3) * sizeof(int) +
                     ((size_t)kProjRI * W + kProjPad) * esz;
  if (lds > 64 * 1024) return hipErrorNotSupported;
  const bool outer = X0.active;
  if (outer && h.s1n < m0 * n1 * (int64_t)n2) return hipErrorNotSupported;
  double *T = outer ? h.s1 : h.c;
  const Rows r1 = rows_of(X1, 0);
  const dim3 g1(nk1c * nk2c, (unsigned)m0);
  const int LT2 = X2.NT.L;
  // column slices per thread of a staged row (the register prefetch holds
  // kProjRI x NCW values)
  const int ncw = (int)((W + BS - 1) / BS);
  if (ncw > 4) return hipErrorNotSupported;
#define MFA_PI(TQ, NTR, NCW)                                                                       \
  k_proj_inner<TQ, P, kProjRI, NTR, NCW><<<g1, BS, lds, h.stream>>>(                                \
      reinterpret_cast<const TQ *>(q), T, m1, m2, n1, n2, K1C, r1, X2.NT.col, X2.NT.len, X2.NT.val, \
      LT2, maxrows1)
#define MFA_PI2(NTR)                                   \
  if (ncw <= 2) {                                      \
    if (f32) MFA_PI(float, NTR, 2);                    \
    else MFA_PI(double, NTR, 2);                       \
  } else {                                             \
    if (f32) MFA_PI(float, NTR, 4);                    \
    else MFA_PI(double, NTR, 4);                       \
  }
  if (LT2 <= 12) {
    MFA_PI2(12)
  } else if (LT2 <= 24) {
    MFA_PI2(24)
  } else if (LT2 <= 48) {
    MFA_PI2(48)
  } else {
    return hipErrorNotSupported;
  }
#undef MFA_PI2
#undef MFA_PI
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !outer) return e;
  const int64_t J = (int64_t)n1 * n2;
  const int K0C = pick_chunk((int64_t)nblk(J, 256), n0, 8);
  int maxrows0 = 0;
  for (int c = 0; c < (int)nblk(n0, K0C); ++c)
    maxrows0 = (int)std::max<int64_t>(maxrows0, rows_of_chunk(m0, n0, c * K0C, std::min(n0, c * K0C + K0C)));
  const size_t lds0 = (size_t)maxrows0 * ((P + 1) * sizeof(double) + sizeof(int));
  if (lds0 > 64 * 1024) return hipErrorInvalidValue;
  const dim3 g0(nblk(J, 256), nblk(n0, K0C));
  k_proj_outer<P><<<g0, 256, lds0, h.stream>>>(T, h.c, J, n0, K0C, rows_of(X0, 0), maxrows0);
  return hipGetLastError();
}

// Decode to FP32 with axes 1 and 2 on the matrix cores (k_dec_mfma): axis 0
// first into an FP32 intermediate, then the operand tables, then the tiles.
// hipErrorNotSupported when a shape does not fit the kernel's windows (the
// caller then takes the vector kernels): a tile of 16 points of axis 1 must
// see at most 16 control rows, and one of axis 2 at most two aligned tiles of
// 16 control columns.  Scratch (h.s1): the intermediate, then the tables.
template <int P>
hipError_t decode_mfma(Handle &h, float *out, const int r[3]) {
  const Axis &X0 = h.ax[0], &X1 = h.ax[1], &X2 = h.ax[2];
  const int64_t m0 = X0.active ? X0.m : 1, m1 = X1.m, m2 = X2.m;
  const int n1 = X1.n, n2 = X2.n;
  if (getenv("MFA_VECTOR_DECODE")) return hipErrorNotSupported;
  if ((int64_t)n1 * n2 >= (int64_t)1 << 31) return hipErrorNotSupported;
  // host copy of the span rule: span(i) = min(n-1, p + floor(i (n-p) / (m-1)))
  auto span = [](int64_t i, int64_t m, int n) {
    return (int)std::min<int64_t>(n - 1, P + i * (n - P) / (m - 1));
  };
  const int nt1 = (int)((m1 + 15) / 16), nt2 = (int)((m2 + 15) / 16);
  int ext1 = 0;
  for (int I = 0; I < nt1; ++I)
    ext1 = std::max(ext1, span(std::min<int64_t>(16 * (int64_t)I + 15, m1 - 1), m1, n1) -
                              span(16 * (int64_t)I, m1, n1) + P + 1);
  // one wave holds the U tiles of all of axis 2's control columns in registers
  if (ext1 > 16 || n2 > 256) return hipErrorNotSupported;
  for (int J2 = 0; J2 < nt2; ++J2) {
    const int lo = span(16 * (int64_t)J2, m2, n2) - P;
    const int hi = span(std::min<int64_t>(16 * (int64_t)J2 + 15, m2 - 1), m2, n2);
    if (hi / 16 - lo / 16 > 1) return hipErrorNotSupported;
  }
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t tbytes = X0.active ? up((size_t)m0 * n1 * n2 * sizeof(float)) : 0;
  const size_t w1b = up((size_t)nt1 * 256 * sizeof(float)), w2b = up((size_t)nt2 * 512 * sizeof(float));
  const int ntk = (n2 + 15) / 16;
  const size_t lds = (size_t)nt2 * 128 * 16 + (size_t)(nt2 + ntk + 1) * sizeof(int);
  if (lds > 64 * 1024) return hipErrorNotSupported;
  const size_t need = tbytes + w1b + w2b + up((size_t)nt1 * sizeof(int)) + up((size_t)nt2 * sizeof(int)) +
                      up((size_t)(ntk + 1) * sizeof(int));
  if ((size_t)h.s1n * sizeof(double) < need) return hipErrorNotSupported;
  char *base = reinterpret_cast<char *>(h.s1);
  float *tmid = reinterpret_cast<float *>(base);
  float *w1t = reinterpret_cast<float *>(base + tbytes);
  float *w2t = reinterpret_cast<float *>(base + tbytes + w1b);
  int *klo1 = reinterpret_cast<int *>(base + tbytes + w1b + w2b);
  int *j0n = reinterpret_cast<int *>(base + tbytes + w1b + w2b + up((size_t)nt1 * sizeof(int)));
  int *j2beg = reinterpret_cast<int *>(base + tbytes + w1b + w2b + up((size_t)nt1 * sizeof(int)) +
                                       up((size_t)nt2 * sizeof(int)));
  hipError_t e;
  if (X0.active) {
    const int64_t J = (int64_t)n1 * n2;
    const int I0C = 64;
    const dim3 g0(nblk(J, 256), nblk(m0, I0C));
    const size_t lds0 = (size_t)I0C * ((P + 1) * sizeof(double) + sizeof(int));
    k_dec_outer<P, float><<<g0, 256, lds0, h.stream>>>(h.P, tmid, J, I0C, rows_of(X0, r[0]));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const Rows r1 = rows_of(X1, r[1]), r2 = rows_of(X2, r[2]);
  const int64_t ntab = (int64_t)nt1 * 64 + (int64_t)nt2 * 128 + ntk + 1;
  k_dec_tab<P><<<nblk(ntab, 256), 256, 0, h.stream>>>(r1, r2, nt1, nt2, ntk, w1t, klo1, w2t, j0n, j2beg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 8 waves per workgroup share the staged N_2 table
  const int wpb = (int)std::min<int64_t>(8, nt1);
  const dim3 g1(nblk(nt1, wpb), (unsigned)m0);
  const bool v4 = m2 % 4 == 0;
#define MFA_DM(TI, SRC, NTK_)                                                                    \
  do {                                                                                           \
    if (v4)                                                                                      \
      k_dec_mfma<TI, true, NTK_><<<g1, 64 * wpb, lds, h.stream>>>(SRC, out, m1, m2, n1, n2, nt1, \
                                                                  nt2, w1t, klo1, w2t, j0n, j2beg); \
    else                                                                                         \
      k_dec_mfma<TI, false, NTK_><<<g1, 64 * wpb, lds, h.stream>>>(SRC, out, m1, m2, n1, n2, nt1, \
                                                                   nt2, w1t, klo1, w2t, j0n, j2beg); \
  } while (0)
#define MFA_DM_NTK(TI, SRC)                    \
  if (ntk <= 4) MFA_DM(TI, SRC, 4);            \
  else if (ntk <= 8) MFA_DM(TI, SRC, 8);       \
  else if (ntk <= 12) MFA_DM(TI, SRC, 12);     \
  else MFA_DM(TI, SRC, 16);
  if (X0.active) {
    MFA_DM_NTK(float, tmid);
  } else {
    MFA_DM_NTK(double, h.P);
  }
#undef MFA_DM_NTK
#undef MFA_DM
  return hipGetLastError();
}

template <int P>
hipError_t decode_p(Handle &h, void *out, bool f32, const int r[3], unsigned long long *rs) {
  const Axis &X0 = h.ax[0], &X1 = h.ax[1], &X2 = h.ax[2];
  const int64_t m0 = X0.m, m1 = X1.m, m2 = X2.m;
  const int n1 = X1.n, n2 = X2.n;
  if (n2 > 256) return hipErrorNotSupported;
  const int BS = m2 >= 256 || n2 > 128 ? 256 : (int)std::max<int64_t>(64, ((std::max<int64_t>(m2, n2) + 63) / 64) * 64);
  const int IS = (int)((m2 + BS - 1) / BS);
  if (IS > 4) return hipErrorNotSupported;
  if (f32 && !rs) {
    hipError_t e = decode_mfma<P>(h, reinterpret_cast<float *>(out), r);
    if (e != hipErrorNotSupported) return e;
  }
  const double *src = h.P;
  if (X0.active) {
    if (h.s1n < m0 * n1 * (int64_t)n2) return hipErrorNotSupported;
    const int64_t J = (int64_t)n1 * n2;
    const int I0C = 64;
    const dim3 g0(nblk(J, 256), nblk(m0, I0C));
    const size_t lds0 = (size_t)I0C * ((P + 1) * sizeof(double) + sizeof(int));
    k_dec_outer<P, double><<<g0, 256, lds0, h.stream>>>(h.P, h.s1, J, I0C, rows_of(X0, r[0]));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    src = h.s1;
  }
  int I1C = 64;
  while (I1C > 8 && m0 * (int64_t)nblk(m1, I1C) < 2048) I1C /= 2;
  const dim3 g1(nblk(m1, I1C), (unsigned)m0);
  const size_t lds = (size_t)kDecRI * n2 * sizeof(double) + (size_t)I1C * ((P + 1) * sizeof(double) + sizeof(int));
  const Rows r1 = rows_of(X1, r[1]), r2 = rows_of(X2, r[2]);
#define MFA_DI(TO, IS_)                                                                          \
  if (rs)                                                                                        \
    k_dec_inner<TO, P, kDecRI, IS_, true><<<g1, BS, lds, h.stream>>>(                            \
        src, reinterpret_cast<TO *>(out), m1, m2, n1, n2, I1C, r1, r2, rs);                      \
  else                                                                                           \
    k_dec_inner<TO, P, kDecRI, IS_, false><<<g1, BS, lds, h.stream>>>(                           \
        src, reinterpret_cast<TO *>(out), m1, m2, n1, n2, I1C, r1, r2, nullptr)
  if (IS == 1) {
    if (f32) { MFA_DI(float, 1); }
    else { MFA_DI(double, 1); }
  } else if (IS == 2) {
    if (f32) { MFA_DI(float, 2); }
    else { MFA_DI(double, 2); }
  } else {
    if (f32) { MFA_DI(float, 4); }
    else { MFA_DI(double, 4); }
  }
#undef MFA_DI
  return hipGetLastError();
}

}  // namespace

bool grid_pass_ok(const Handle &h) { return h.ax[1].active && h.ax[2].active && h.p >= 1 && h.p <= 6; }

hipError_t launch_project_grid(Handle &h, const void *q, bool f32) {
  switch (h.p) {
    case 1: return project_p<1>(h, q, f32);
    case 2: return project_p<2>(h, q, f32);
    case 3: return project_p<3>(h, q, f32);
    case 4: return project_p<4>(h, q, f32);
    case 5: return project_p<5>(h, q, f32);
    case 6: return project_p<6>(h, q, f32);
    default: return hipErrorNotSupported;
  }
}

hipError_t launch_decode_grid(Handle &h, void *out, bool f32, const int r[3],
                              unsigned long long *rs) {
  switch (h.p) {
    case 1: return decode_p<1>(h, out, f32, r, rs);
    case 2: return decode_p<2>(h, out, f32, r, rs);
    case 3: return decode_p<3>(h, out, f32, r, rs);
    case 4: return decode_p<4>(h, out, f32, r, rs);
    case 5: return decode_p<5>(h, out, f32, r, rs);
    case 6: return decode_p<6>(h, out, f32, r, rs);
    default: return hipErrorNotSupported;
  }
}

}  // namespace mfa
