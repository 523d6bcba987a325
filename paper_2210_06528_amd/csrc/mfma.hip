// Mixed-precision Schwarz correction on the matrix cores (MFMA, BF16 inputs,
// FP32 accumulation).  Along each axis the weighted additive-Schwarz operator
//   M_a = sum_b w_b R_b^T (N_b^T N_b)^{-1} R_b
// is a dense block-banded matrix (the local inverses of overlapping
// subdomains), so one correction pass is a banded GEMM:
//   axes 0/1 (strided)   : OUT[k][i] = sum_j M_a[k][j] IN[j][i]   (A = M_a, B = IN)
//   axis 2 (contiguous)  : OUT[o][k] = sum_j IN[o][j] M_a[k][j]   (A = IN,  B = M_a^T)
// with v_mfma_f32_16x16x32_bf16 tiles (operands split hi+lo, see below) and
// FP32 accumulation.  The K range of every 16-row tile of M_a is restricted to
// its band.  The residual feeding these passes is the float64 residual of the
// normal equations rounded to FP32, so the sweep is an iterative refinement on
// the float64 residual.
#include <hip/hip_bf16.h>

#include "mfa_internal.hpp"

namespace mfa {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// MFMA 16x16x32 operand lane layout (checked against a CPU product):
//   A (16 x 32): lane l holds row l%16, k = 8*(l/16) .. 8*(l/16)+7
//   B (32 x 16): lane l holds col l%16, the same k range
//   C (16 x 16): lane l holds rows 4*(l/16)+v (v = 0..3), col l%16

__device__ __forceinline__ bf16x8 load8(const __hip_bfloat16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ void slot_max_m(unsigned long long *slots, int slot, double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) {
    const unsigned copy =
        (blockIdx.x * 7u + blockIdx.y * 131u + blockIdx.z * 1031u + (threadIdx.x >> 6)) % kSlotCopies;
    atomicMax(slots + (size_t)slot * kSlotCopies + copy, (unsigned long long)__double_as_longlong(v));
  }
}

// Operands are split into two BF16 terms, x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (about 16 significant bits together), and every product
// accumulates hi*hi + hi*lo + lo*hi in FP32 ("bf16x3"): plain BF16 rounding of
// the correction operator is amplified by the condition number of the local
// normal matrices on every axis pass and ruins the Schwarz contraction.
__device__ __forceinline__ void split_bf16(float x, __hip_bfloat16 &hi, __hip_bfloat16 &lo) {
  hi = __float2bfloat16(x);
  lo = __float2bfloat16(x - __bfloat162float(hi));
}

__device__ __forceinline__ floatx4 mfma3(const bf16x8 &ahi, const bf16x8 &alo, const bf16x8 &bhi,
                                         const bf16x8 &blo, floatx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
  return acc;
}

constexpr int kIT = 32;    // columns per workgroup on the strided axes
constexpr int kStage = 16; // staging loads per thread issued before the first wait
constexpr int kPre = 4;    // K chunks of a tile's M fragments requested up front

// Strided axis: the array is [outer][n][inner] (FP32); workgroup = (one outer
// index, kIT columns of inner), all n output rows.  IN[:, i0:i0+kIT] is staged
// in LDS transposed and split (Thi/Tlo[i][j], j contiguous) so a B fragment is
// one 16-byte LDS read.  Wave w computes row tiles w, w+4, ...; MODE 0 stores
// FP32, MODE 1 adds into the float64 control points and reduces max |corr|.
template <int MODE>
__global__ void __launch_bounds__(256) k_mfma_strided(const float *__restrict__ in,
                                                      float *__restrict__ out,
                                                      double *__restrict__ pc, int n, int64_t inner,
                                                      int npad, const __hip_bfloat16 *__restrict__ Mhi,
                                                      const __hip_bfloat16 *__restrict__ Mlo,
                                                      const int *__restrict__ klo,
                                                      const int *__restrict__ knc,
                                                      unsigned long long *slots) {
  extern __shared__ __hip_bfloat16 T[];   // hi: [kIT][npad + 8], then lo
  const int ld = npad + 8;
  __hip_bfloat16 *Thi = T, *Tlo = T + kIT * ld;
  const int64_t o = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * kIT;
  // staging: kStage loads per thread in flight before the first wait
  for (int e0 = 0; e0 < npad * kIT; e0 += 256 * kStage) {
    float v[kStage];
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = e0 + threadIdx.x + 256 * r;
      const int j = e / kIT, ii = e - j * kIT;
      v[r] = (e < npad * kIT && j < n && i0 + ii < inner) ? in[(o * n + j) * inner + i0 + ii] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = e0 + threadIdx.x + 256 * r;
      const int j = e / kIT, ii = e - j * kIT;
      if (e < npad * kIT) split_bf16(v[r], Thi[ii * ld + j], Tlo[ii * ld + j]);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles = (n + 15) >> 4;
  double dmax = 0.0;
  for (int t = w; t < ntiles; t += 4) {
    floatx4 acc[kIT / 16];
#pragma unroll
    for (int s = 0; s < kIT / 16; ++s) acc[s] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int lo = klo[t], nc = knc[t];
    const int64_t moff = (int64_t)(16 * t + r16) * npad + 8 * kq;
    // the tile's M fragments (all K chunks) are requested before the first MFMA
    bf16x8 ahi[kPre], alo[kPre];
#pragma unroll
    for (int c = 0; c < kPre; ++c) {
      if (c < nc) {
        ahi[c] = load8(Mhi + moff + lo + 32 * c);
        alo[c] = load8(Mlo + moff + lo + 32 * c);
      }
    }
#pragma unroll
    for (int c = 0; c < kPre; ++c) {
      if (c < nc) {
        const int j0 = lo + 32 * c;
#pragma unroll
        for (int s = 0; s < kIT / 16; ++s) {
          const int toff = (16 * s + r16) * ld + j0 + 8 * kq;
          acc[s] = mfma3(ahi[c], alo[c], load8(Thi + toff), load8(Tlo + toff), acc[s]);
        }
      }
    }
    for (int c = kPre; c < nc; ++c) {
      const int j0 = lo + 32 * c;
      const bf16x8 bh = load8(Mhi + moff + j0), bl = load8(Mlo + moff + j0);
#pragma unroll
      for (int s = 0; s < kIT / 16; ++s) {
        const int toff = (16 * s + r16) * ld + j0 + 8 * kq;
        acc[s] = mfma3(bh, bl, load8(Thi + toff), load8(Tlo + toff), acc[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < kIT / 16; ++s) {
      const int64_t i = i0 + 16 * s + r16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * t + 4 * kq + v;
        if (k < n && i < inner) {
          const int64_t idx = (o * n + k) * inner + i;
          if (MODE == 0) {
            out[idx] = acc[s][v];
          } else {
            const double d = (double)acc[s][v];
            pc[idx] += d;
            dmax = fmax(dmax, fabs(d));
          }
        }
      }
    }
  }
  if (MODE == 1) slot_max_m(slots, kSlotMaxDP, dmax);
}

// Contiguous axis: the array is [nlines][n] (FP32); workgroup = 16*nw lines
// staged in LDS (split), wave w holds lines 16w..16w+15 and computes every
// row tile of M_a for them.
template <int MODE>
__global__ void __launch_bounds__(256) k_mfma_contig(const float *__restrict__ in,
                                                     float *__restrict__ out,
                                                     double *__restrict__ pc, int n, int64_t nlines,
                                                     int npad, const __hip_bfloat16 *__restrict__ Mhi,
                                                     const __hip_bfloat16 *__restrict__ Mlo,
                                                     const int *__restrict__ klo,
                                                     const int *__restrict__ knc,
                                                     unsigned long long *slots) {
  extern __shared__ __hip_bfloat16 Ls[];   // hi: [lpw][npad + 8], then lo
  const int ld = npad + 8;
  const int lpw = blockDim.x / 4;          // 16 lines per wave
  __hip_bfloat16 *Lhi = Ls, *Llo = Ls + lpw * ld;
  const int64_t l0 = (int64_t)blockIdx.x * lpw;
  const int nt = blockDim.x;
  for (int e0 = 0; e0 < npad * lpw; e0 += nt * kStage) {
    float v[kStage];
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = e0 + threadIdx.x + nt * r;
      const int li = e / npad, j = e - li * npad;
      v[r] = (e < npad * lpw && j < n && l0 + li < nlines) ? in[(l0 + li) * n + j] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int e = e0 + threadIdx.x + nt * r;
      const int li = e / npad, j = e - li * npad;
      if (e < npad * lpw) split_bf16(v[r], Lhi[li * ld + j], Llo[li * ld + j]);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles = (n + 15) >> 4;
  const int aoff = (16 * w + r16) * ld + 8 * kq;
  double dmax = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
    const int lo = klo[t], nc = knc[t];
    const int64_t moff = (int64_t)(16 * t + r16) * npad + 8 * kq;
    bf16x8 bhi[kPre], blo[kPre];
#pragma unroll
    for (int c = 0; c < kPre; ++c) {
      if (c < nc) {
        bhi[c] = load8(Mhi + moff + lo + 32 * c);
        blo[c] = load8(Mlo + moff + lo + 32 * c);
      }
    }
#pragma unroll
    for (int c = 0; c < kPre; ++c) {
      if (c < nc) {
        const int j0 = lo + 32 * c;
        acc = mfma3(load8(Lhi + aoff + j0), load8(Llo + aoff + j0), bhi[c], blo[c], acc);
      }
    }
    for (int c = kPre; c < nc; ++c) {
      const int j0 = lo + 32 * c;
      acc = mfma3(load8(Lhi + aoff + j0), load8(Llo + aoff + j0), load8(Mhi + moff + j0),
                  load8(Mlo + moff + j0), acc);
    }
    const int k = 16 * t + r16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t line = l0 + 16 * w + 4 * kq + v;
      if (k < n && line < nlines) {
        const int64_t idx = line * n + k;
        if (MODE == 0) {
          out[idx] = acc[v];
        } else {
          const double d = (double)acc[v];
          pc[idx] += d;
          dmax = fmax(dmax, fabs(d));
        }
      }
    }
  }
  if (MODE == 1) slot_max_m(slots, kSlotMaxDP, dmax);
}

// dense split-BF16 copy of M_a (rows padded to a multiple of 16 with zeros,
// columns to npad) from its float64 row table
__global__ void k_tab_Mbf16(int n, int nrows, int npad, Ell M, __hip_bfloat16 *Mhi,
                            __hip_bfloat16 *Mlo) {
  const int k = blockIdx.x;
  if (k >= nrows) return;
  for (int j = threadIdx.x; j < npad; j += blockDim.x) {
    Mhi[(int64_t)k * npad + j] = __float2bfloat16(0.0f);
    Mlo[(int64_t)k * npad + j] = __float2bfloat16(0.0f);
  }
  __syncthreads();
  if (k >= n) return;
  const int len = M.len[k];
  for (int q = threadIdx.x; q < len; q += blockDim.x) {
    const int64_t o = (int64_t)k * npad + M.col[(int64_t)k * M.L + q];
    const double v = M.val[(int64_t)k * M.L + q];
    const __hip_bfloat16 hi = __float2bfloat16((float)v);
    Mhi[o] = hi;
    Mlo[o] = __float2bfloat16((float)(v - (double)__bfloat162float(hi)));
  }
}

// K range of every 16-row tile: [lo, lo + 32*nc) covers the band of its rows,
// lo a multiple of 8 (16-byte aligned fragments)
__global__ void k_tab_ktiles(int n, Ell M, int *klo, int *knc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (n + 15) / 16) return;
  int lo = 1 << 30, hi = 0;
  for (int k = 16 * t; k < min(n, 16 * t + 16); ++k) {
    const int c0 = M.col[(int64_t)k * M.L], len = M.len[k];
    lo = min(lo, c0);
    hi = max(hi, c0 + len);
  }
  lo &= ~7;
  klo[t] = lo;
  knc[t] = (hi - lo + 31) / 32;
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// LDS of the strided kernel; the contiguous kernel picks its lines per
// workgroup (64, 32 or 16) to stay within 64 KB
size_t mfma_lds(int npad) { return sizeof(__hip_bfloat16) * 2 * kIT * (size_t)(npad + 8); }

static int contig_lines(int npad) {
  for (int lpw = 64; lpw >= 16; lpw /= 2)
    if (sizeof(__hip_bfloat16) * 2 * (size_t)lpw * (npad + 8) <= 64 * 1024) return lpw;
  return 0;
}

bool mfma_fits(int npad) { return mfma_lds(npad) <= 64 * 1024 && contig_lines(npad) > 0; }

hipError_t setup_mfma(Handle *h, int ia, hipStream_t st) {
  Axis &X = h->ax[ia];
  const int nrows = (X.n + 15) / 16 * 16;
  __hip_bfloat16 *Mhi = reinterpret_cast<__hip_bfloat16 *>(X.d_Mb);
  __hip_bfloat16 *Mlo = Mhi + (int64_t)nrows * X.npad;
  k_tab_Mbf16<<<nrows, 128, 0, st>>>(X.n, nrows, X.npad, X.M, Mhi, Mlo);
  k_tab_ktiles<<<nblk((X.n + 15) / 16, 64), 64, 0, st>>>(X.n, X.M, X.d_klo, X.d_knc);
  return hipGetLastError();
}

hipError_t launch_mfma_correct(Handle &h, int axis, const float *in, float *out, bool add) {
  const Axis &X = h.ax[axis];
  const int n = X.n;
  const int nrows = (n + 15) / 16 * 16;
  const __hip_bfloat16 *Mhi = reinterpret_cast<const __hip_bfloat16 *>(X.d_Mb);
  const __hip_bfloat16 *Mlo = Mhi + (int64_t)nrows * X.npad;
  if (axis == 2) {
    const int64_t nlines = (int64_t)h.ax[0].n * h.ax[1].n;
    const int lpw = contig_lines(X.npad);
    const size_t lds = sizeof(__hip_bfloat16) * 2 * (size_t)lpw * (X.npad + 8);
    const unsigned grid = nblk(nlines, lpw);
    const int threads = 4 * lpw;
    if (add)
      k_mfma_contig<1><<<grid, threads, lds, h.stream>>>(in, out, h.P, n, nlines, X.npad, Mhi, Mlo,
                                                         X.d_klo, X.d_knc, h.slots);
    else
      k_mfma_contig<0><<<grid, threads, lds, h.stream>>>(in, out, h.P, n, nlines, X.npad, Mhi, Mlo,
                                                         X.d_klo, X.d_knc, h.slots);
  } else {
    const int64_t outer = axis == 0 ? 1 : h.ax[0].n;
    const int64_t inner = axis == 0 ? (int64_t)h.ax[1].n * h.ax[2].n : h.ax[2].n;
    const dim3 grid(nblk(inner, kIT), (unsigned)outer);
    const size_t lds = mfma_lds(X.npad);
    if (add)
      k_mfma_strided<1><<<grid, 256, lds, h.stream>>>(in, out, h.P, n, inner, X.npad, Mhi, Mlo,
                                                      X.d_klo, X.d_knc, h.slots);
    else
      k_mfma_strided<0><<<grid, 256, lds, h.stream>>>(in, out, h.P, n, inner, X.npad, Mhi, Mlo,
                                                      X.d_klo, X.d_knc, h.slots);
  }
  return hipGetLastError();
}

}  // namespace mfa
