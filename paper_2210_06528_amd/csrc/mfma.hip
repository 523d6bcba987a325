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
//
// In 3-D the axis-2 and axis-1 passes run as one kernel (k_mfma_fused21)
// whose intermediate stays in LDS; the axis-0 pass adds into the control
// points.  Every pass stages its input in LDS split into BF16 halves, eight
// values per 16-byte store (a 2-byte store per value made the staging
// LDS-bank-bound), so that an MFMA operand fragment is one 16-byte read.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <vector>

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

// The workgroup's max of v, one atomic on one copy of the slot: wavefront
// maxima through LDS, then thread 0.  Every thread of the workgroup must
// call it (it has a barrier).  One atomic per workgroup instead of one per
// wavefront: the atomics on a slot's copies queue at L2, and at the end of a
// kernel whose workgroups all finish together that queue is the kernel's tail.
__device__ __forceinline__ void block_slot_max_m(unsigned long long *slots, int slot, double v) {
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
constexpr int kPre = 4;    // K chunks of a tile's M fragments requested up front

// Split 8 values into BF16 hi/lo and store each half as one 16-byte LDS write.
__device__ __forceinline__ void store_split8(const float (&v)[8], __hip_bfloat16 *hi,
                                             __hip_bfloat16 *lo) {
  __hip_bfloat16 hb[8], lb[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) split_bf16(v[q], hb[q], lb[q]);
  bf16x8 hv, lv;
  __builtin_memcpy(&hv, hb, sizeof(hv));
  __builtin_memcpy(&lv, lb, sizeof(lv));
  *reinterpret_cast<bf16x8 *>(hi) = hv;
  *reinterpret_cast<bf16x8 *>(lo) = lv;
}

// Stage in[j * inner + i0 + ii] (rows j < n, zeros up to npad; columns
// ii < kIT, zeros past inner) transposed and split: Thi/Tlo[ii * ld + j].  A
// thread takes column ii and blocks of 8 rows (the loads coalesce across the
// kIT columns, two blocks in flight); each block is one 16-byte write per
// half (rows ld = npad + 8 elements apart put 16 lanes' groups in distinct
// banks).  256 threads.
__device__ __forceinline__ void stage_transposed(const float *__restrict__ in, int64_t inner, int n,
                                                 int npad, int64_t i0, __hip_bfloat16 *Thi,
                                                 __hip_bfloat16 *Tlo, int ld) {
  constexpr int BPP = 256 / kIT;   // row blocks per pass of the workgroup
  const int ii = threadIdx.x % kIT;
  const int nb8 = npad / 8;
  const bool colok = i0 + ii < inner;
  for (int b0 = threadIdx.x / kIT; b0 < nb8; b0 += 2 * BPP) {
    float v[2][8];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int jb = b0 + hh * BPP;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = 8 * jb + q;
        v[hh][q] = (jb < nb8 && j < n && colok) ? in[(int64_t)j * inner + i0 + ii] : 0.f;
      }
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int jb = b0 + hh * BPP;
      if (jb < nb8) store_split8(v[hh], Thi + ii * ld + 8 * jb, Tlo + ii * ld + 8 * jb);
    }
  }
}

// Stage nl lines of in (line li at in + li * n; columns j < n, zeros up to
// npad; lines past nl zero) split row-wise: Lhi/Llo[li * ld + j], in blocks of
// 8 columns, two per thread in flight, 16-byte loads when VEC (rows 16-byte
// aligned).  nt threads.
template <bool VEC>
__device__ __forceinline__ void stage_rows(const float *__restrict__ in, int n, int npad, int lines,
                                           int nl, __hip_bfloat16 *Lhi, __hip_bfloat16 *Llo, int ld,
                                           int nt) {
  const int nbw = npad / 8, nblk = lines * nbw;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 2 * nt) {
    float v[2][8];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int bi = b0 + hh * nt;
      const int li = bi / nbw, j0 = 8 * (bi - li * nbw);
      const bool ok = bi < nblk && li < nl;
      const float *src = in + (int64_t)(ok ? li : 0) * n + (ok ? j0 : 0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (VEC && ok && j0 + 4 * u + 3 < n) {
          const float4 f = *reinterpret_cast<const float4 *>(src + 4 * u);
          v[hh][4 * u] = f.x;
          v[hh][4 * u + 1] = f.y;
          v[hh][4 * u + 2] = f.z;
          v[hh][4 * u + 3] = f.w;
        } else {
#pragma unroll
          for (int q = 4 * u; q < 4 * u + 4; ++q) v[hh][q] = (ok && j0 + q < n) ? src[q] : 0.f;
        }
      }
    }
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int bi = b0 + hh * nt;
      if (bi < nblk) {
        const int li = bi / nbw, j0 = 8 * (bi - li * nbw);
        store_split8(v[hh], Lhi + li * ld + j0, Llo + li * ld + j0);
      }
    }
  }
}

// Apply M_a (rows from global, split) to the kIT staged columns Thi/Tlo
// ([kIT][ld], contraction index contiguous) of outer index o: OUT[o][k][i0+ii]
// for every row k; MODE 0 stores FP32, MODE 1 adds into the float64 control
// points and keeps max |correction| in dmax.  Waves take row tiles w, w+4, ...
template <int MODE>
__device__ __forceinline__ void strided_apply(const __hip_bfloat16 *Thi, const __hip_bfloat16 *Tlo, int ld,
                                              float *__restrict__ out, double *__restrict__ pc, int n,
                                              int64_t inner, int npad, int64_t o, int64_t i0,
                                              const __hip_bfloat16 *__restrict__ Mhi,
                                              const __hip_bfloat16 *__restrict__ Mlo,
                                              const int *__restrict__ klo, const int *__restrict__ knc,
                                              double &dmax) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles = (n + 15) >> 4;
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
    // MODE 1: the control points this tile updates are requested before the
    // products too
    double pold[kIT / 16][4];
    if (MODE == 1) {
#pragma unroll
      for (int s = 0; s < kIT / 16; ++s) {
        const int64_t i = i0 + 16 * s + r16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = 16 * t + 4 * kq + v;
          pold[s][v] = (k < n && i < inner) ? pc[(o * n + k) * inner + i] : 0.0;
        }
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
            pc[idx] = pold[s][v] + d;
            dmax = fmax(dmax, fabs(d));
          }
        }
      }
    }
  }
}

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
  stage_transposed(in + o * n * inner, inner, n, npad, i0, Thi, Tlo, ld);
  __syncthreads();
  double dmax = 0.0;
  strided_apply<MODE>(Thi, Tlo, ld, out, pc, n, inner, npad, o, i0, Mhi, Mlo, klo, knc, dmax);
  if (MODE == 1) block_slot_max_m(slots, kSlotMaxDP, dmax);
}

// Axis-0 pass that adds into the control points (outer = 1), for n <= 64 *
// kPT: every wave's control points (kPT row tiles) are requested at the
// start, with the staging loads, instead of one HBM round trip per tile after
// the products (they hold 64 registers: two waves per SIMD, still faster).
// Loads use clamped in-bounds indices; the same MFMA sequence as
// k_mfma_strided<1>.
constexpr int kPT = 4;
__global__ void __launch_bounds__(256) k_mfma_axis0_add(const float *__restrict__ in,
                                                        double *__restrict__ pc, int n, int64_t inner,
                                                        int npad, const __hip_bfloat16 *__restrict__ Mhi,
                                                        const __hip_bfloat16 *__restrict__ Mlo,
                                                        const int *__restrict__ klo,
                                                        const int *__restrict__ knc,
                                                        unsigned long long *slots) {
  extern __shared__ __hip_bfloat16 T[];   // hi: [kIT][npad + 8], then lo
  const int ld = npad + 8;
  __hip_bfloat16 *Thi = T, *Tlo = T + kIT * ld;
  const int64_t i0 = (int64_t)blockIdx.x * kIT;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles = (n + 15) >> 4;
  double pold[kPT][kIT / 16][4];
#pragma unroll
  for (int j = 0; j < kPT; ++j) {
    const int t = w + 4 * j;
#pragma unroll
    for (int s = 0; s < kIT / 16; ++s) {
      const int64_t i = min(i0 + 16 * s + r16, inner - 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = min(16 * t + 4 * kq + v, n - 1);
        pold[j][s][v] = pc[(int64_t)k * inner + i];
      }
    }
  }
  stage_transposed(in, inner, n, npad, i0, Thi, Tlo, ld);
  __syncthreads();
  double dmax = 0.0;
#pragma unroll
  for (int j = 0; j < kPT; ++j) {
    const int t = w + 4 * j;
    if (t < ntiles) {
      floatx4 acc[kIT / 16];
#pragma unroll
      for (int s = 0; s < kIT / 16; ++s) acc[s] = floatx4{0.f, 0.f, 0.f, 0.f};
      const int lo = klo[t], nc = knc[t];
      const int64_t moff = (int64_t)(16 * t + r16) * npad + 8 * kq;
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
            const double d = (double)acc[s][v];
            pc[(int64_t)k * inner + i] = pold[j][s][v] + d;
            dmax = fmax(dmax, fabs(d));
          }
        }
      }
    }
  }
  block_slot_max_m(slots, kSlotMaxDP, dmax);
}

// Contiguous axis: the array is [nlines][n] (FP32); workgroup = 16*nw lines
// staged in LDS (split), wave w holds lines 16w..16w+15 and computes every
// row tile of M_a for them.
template <int MODE, bool VEC>
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
  stage_rows<VEC>(in + l0 * n, n, npad, lpw, (int)min((int64_t)lpw, nlines - l0), Lhi, Llo, ld, nt);
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
  if (MODE == 1) block_slot_max_m(slots, kSlotMaxDP, dmax);
}

// Axes 2 and 1 of the correction in one pass (mode 0): a workgroup takes one
// x-plane o and a block of kIT outputs k2.  Phase 1 applies M_2 to the
// plane's lines, 32 at a time (staged split in LDS, only the columns the two
// output tiles need), and keeps the result split in LDS, transposed as the
// strided pass stages its input; phase 2 is that strided pass along axis 1.
// Every output takes the same MFMA sequence as the two separate passes, so
// the result is the same; the intermediate never goes through HBM.
// The grid is one-dimensional, nb2 blocks per plane: workgroups are dealt to
// the 8 XCDs round-robin, and the renumbering gives each XCD a contiguous run
// of planes, so the blocks of one plane (whose column ranges overlap) share an
// L2.  The M_2 fragments of a wave's tile are loaded once; the next two
// chunks of lines are in flight in registers while the current one is
// multiplied.  At most 168 registers per lane (three waves per SIMD, as many workgroups per CU
// as the LDS holds).
// NCH > 0: the plane has exactly NCH chunks of 32 lines (n1 <= 32 NCH) and
// the chunk loop is unrolled, so the compiler counts the outstanding loads
// of each chunk exactly; NCH = 0 loops over the chunks at run time (the
// waits at the loop head then also cover the later chunk's loads).
template <bool VEC, int NCH>
__global__ void __launch_bounds__(256, 3) k_mfma_fused21(const float *__restrict__ in, float *__restrict__ out,
                                                      int n1, int n2, int npad1, int npad2,
                                                      const __hip_bfloat16 *__restrict__ M1hi,
                                                      const __hip_bfloat16 *__restrict__ M1lo,
                                                      const int *__restrict__ klo1,
                                                      const int *__restrict__ knc1,
                                                      const __hip_bfloat16 *__restrict__ M2hi,
                                                      const __hip_bfloat16 *__restrict__ M2lo,
                                                      const int *__restrict__ klo2,
                                                      const int *__restrict__ knc2, int ldw, int nb2) {
  extern __shared__ __hip_bfloat16 S[];
  const int ld1 = npad1 + 8;
  __hip_bfloat16 *Thi = S, *Tlo = S + kIT * ld1;       // [kIT][ld1]: phase-2 operand
  __hip_bfloat16 *Lhi = S + 2 * kIT * ld1;             // [32 lines][ldw]: phase-1 staging
  __hip_bfloat16 *Llo = Lhi + 32 * ldw;
  const unsigned G = gridDim.x, xcd = blockIdx.x % 8, per = G / 8, rem = G % 8;
  const unsigned lb = xcd * per + min(xcd, rem) + blockIdx.x / 8;
  const int64_t o = lb / nb2;
  const int K2a = (int)(lb % nb2) * kIT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles2 = (n2 + 15) >> 4;
  const int t2a = K2a >> 4;
  const int nt2 = min(2, ntiles2 - t2a);
  int jlo = klo2[t2a], jhi = klo2[t2a] + 32 * knc2[t2a];
  if (nt2 > 1) {
    jlo = min(jlo, klo2[t2a + 1]);
    jhi = max(jhi, klo2[t2a + 1] + 32 * knc2[t2a + 1]);
  }
  const int jw = jhi - jlo;   // a multiple of 8; 32 * jw / 8 <= 512 (checked on the host)
  // wave w: output tile t2a + (w & 1), lines 16*(w >> 1) .. +15 of each chunk
  const bool mine = (w & 1) < nt2;
  const int t = t2a + (w & 1), lbk = w >> 1;
  const int lo2 = mine ? klo2[t] : 0, nc2 = mine ? knc2[t] : 0;
  const int64_t moff = (int64_t)(16 * t + r16) * npad2 + 8 * kq;
  bf16x8 bhi[kPre], blo[kPre];
#pragma unroll
  for (int c = 0; c < kPre; ++c) {
    if (c < nc2) {
      bhi[c] = load8(M2hi + moff + lo2 + 32 * c);
      blo[c] = load8(M2lo + moff + lo2 + 32 * c);
    }
  }
  // rows j1 in [n1, npad1) of the phase-2 operand are zero
  for (int e = threadIdx.x; e < kIT * (npad1 - n1); e += 256) {
    const int ii = e / (npad1 - n1), j = n1 + e % (npad1 - n1);
    Thi[ii * ld1 + j] = __float2bfloat16(0.0f);
    Tlo[ii * ld1 + j] = __float2bfloat16(0.0f);
  }
  const float *plane = in + o * (int64_t)n1 * n2;
  // Phase-1 staging in blocks of 8 consecutive columns of one line (jw is a
  // multiple of 8; at most 2 blocks per thread): read with 16-byte loads when
  // rows are 16-byte aligned (VEC), columns past n2 read as zeros, and each
  // block stored split as one 16-byte write per half.
  const int nbw = jw / 8, nblk32 = 32 * nbw;
  // Two chunks of lines in flight: the loads of chunk l0 + 64 are issued
  // after chunk l0 is staged, so a chunk's data has the products of the
  // chunk before it to arrive.  Every load is issued (indices clamped in
  // bounds) and holds the raw value; the values past the plane are zeroed
  // where the chunk is staged, so that no wait for a chunk's loads comes
  // before its staging (the waits count loads in issue order, and a select
  // right after the load would wait for the later chunk's loads too).
  auto fetch = [&](int l0, float(&v)[2][8]) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int bi = threadIdx.x + 256 * hh;
      const int li = bi / nbw, j0 = jlo + 8 * (bi - li * nbw);
      const float *row = plane + (int64_t)min(l0 + li, n1 - 1) * n2;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (VEC) {
          const int jj = j0 + 4 * u;   // a multiple of 4, as is n2
          const float4 f = *reinterpret_cast<const float4 *>(row + min(jj, n2 - 4));
          v[hh][4 * u] = f.x;
          v[hh][4 * u + 1] = f.y;
          v[hh][4 * u + 2] = f.z;
          v[hh][4 * u + 3] = f.w;
        } else {
#pragma unroll
          for (int q = 4 * u; q < 4 * u + 4; ++q) v[hh][q] = row[min(j0 + q, n2 - 1)];
        }
      }
    }
  };
  auto stage = [&](int l0, const float(&v)[2][8]) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int bi = threadIdx.x + 256 * hh;
      if (bi < nblk32) {
        const int li = bi / nbw, bj = bi - li * nbw, j0 = jlo + 8 * bj;
        const bool ok = l0 + li < n1;
        __hip_bfloat16 hb[8], lb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          // VEC reads 4 values at a time: jj = j0 + 4 (q / 4) < n2 covers them
          const bool okq = ok && (VEC ? j0 + 4 * (q / 4) < n2 : j0 + q < n2);
          split_bf16(okq ? v[hh][q] : 0.f, hb[q], lb[q]);
        }
        bf16x8 hv, lv;
        __builtin_memcpy(&hv, hb, sizeof(hv));
        __builtin_memcpy(&lv, lb, sizeof(lv));
        *reinterpret_cast<bf16x8 *>(Lhi + li * ldw + 8 * bj) = hv;
        *reinterpret_cast<bf16x8 *>(Llo + li * ldw + 8 * bj) = lv;
      }
    }
  };
  auto apply = [&](int l0) {
    if (!mine) return;
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
    const int aoff = (16 * lbk + r16) * ldw + 8 * kq - jlo;
#pragma unroll
    for (int c = 0; c < kPre; ++c) {
      if (c < nc2) {
        const int j0 = lo2 + 32 * c;
        acc = mfma3(load8(Lhi + aoff + j0), load8(Llo + aoff + j0), bhi[c], blo[c], acc);
      }
    }
    // nc2 <= kPre (checked on the host): every K chunk's M_2 fragments are
    // the ones loaded at the start
    const int ii = 16 * (w & 1) + r16;   // output k2 - K2a
    const int j1 = l0 + 16 * lbk + 4 * kq;
    if (j1 + 3 < n1) {   // four consecutive rows: one 8-byte write per half
      __hip_bfloat16 hb[4], lb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) split_bf16(acc[q], hb[q], lb[q]);
      uint2 hv, lv;
      __builtin_memcpy(&hv, hb, sizeof(hv));
      __builtin_memcpy(&lv, lb, sizeof(lv));
      *reinterpret_cast<uint2 *>(Thi + ii * ld1 + j1) = hv;
      *reinterpret_cast<uint2 *>(Tlo + ii * ld1 + j1) = lv;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (j1 + q < n1) split_bf16(acc[q], Thi[ii * ld1 + j1 + q], Tlo[ii * ld1 + j1 + q]);
    }
  };
  // two chunks per trip, so that the buffers swap roles without copies
  float va[2][8], vb[2][8];
  fetch(0, va);
  fetch(32, vb);
  if constexpr (NCH > 0) {
#pragma unroll
    for (int c = 0; c < NCH; c += 2) {
      __syncthreads();   // the previous chunk's staging is consumed
      stage(32 * c, va);
      __syncthreads();
      if (c + 2 < NCH) fetch(32 * c + 64, va);
      apply(32 * c);
      if (c + 1 < NCH) {
        __syncthreads();
        stage(32 * c + 32, vb);
        __syncthreads();
        if (c + 3 < NCH) fetch(32 * c + 96, vb);
        apply(32 * c + 32);
      }
    }
  } else
  for (int l0 = 0; l0 < n1; l0 += 64) {
    __syncthreads();   // the previous chunk's staging is consumed
    stage(l0, va);
    __syncthreads();
    fetch(l0 + 64, va);
    apply(l0);
    if (l0 + 32 >= n1) break;
    __syncthreads();
    stage(l0 + 32, vb);
    __syncthreads();
    fetch(l0 + 96, vb);
    apply(l0 + 32);
  }
  __syncthreads();
  double dmax = 0.0;
  strided_apply<0>(Thi, Tlo, ld1, out, nullptr, n1, n2, npad1, o, K2a, M1hi, M1lo, klo1, knc1, dmax);
}

// dense split-BF16 copy of M_a (rows padded to a multiple of 16 with zeros,
// columns to npad) from its float64 row table; one workgroup per row
__device__ __forceinline__ void tab_Mbf16(int n, int nrows, int npad, Ell M, __hip_bfloat16 *Mhi,
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
// lo a multiple of 8 (16-byte aligned fragments); one thread per tile
__device__ __forceinline__ void tab_ktiles(int n, Ell M, int *klo, int *knc) {
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

// both tables of every active axis in one launch (blockIdx.y: the BF16 rows,
// the tile K ranges; blockIdx.z: the axis)
struct MbArgs {
  int n, nrows, npad;
  Ell M;
  __hip_bfloat16 *Mhi, *Mlo;
  int *klo, *knc;
};

struct MbArgs3 {
  MbArgs a[3];
};

__global__ void k_tab_mfma3(MbArgs3 t) {
  const MbArgs &a = t.a[blockIdx.z];
  if (blockIdx.y == 0)
    tab_Mbf16(a.n, a.nrows, a.npad, a.M, a.Mhi, a.Mlo);
  else
    tab_ktiles(a.n, a.M, a.klo, a.knc);
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

hipError_t setup_mfma_axes(Handle *h, hipStream_t st) {
  MbArgs3 t{};
  int na = 0;
  unsigned gx = 1;
  for (int a = 0; a < 3; ++a) {
    Axis &X = h->ax[a];
    if (!X.active) continue;
    const int nrows = (X.n + 15) / 16 * 16;
    __hip_bfloat16 *Mhi = reinterpret_cast<__hip_bfloat16 *>(X.d_Mb);
    __hip_bfloat16 *Mlo = Mhi + (int64_t)nrows * X.npad;
    t.a[na++] = MbArgs{X.n, nrows, X.npad, X.M, Mhi, Mlo, X.d_klo, X.d_knc};
    gx = std::max(gx, std::max<unsigned>(nrows, nblk((X.n + 15) / 16, 128)));
  }
  if (na == 0) return hipSuccess;
  k_tab_mfma3<<<dim3(gx, 2, na), 128, 0, st>>>(t);
  return hipGetLastError();
}

// Widest column range phase 1 of the fused pass stages for one block of kIT
// outputs along axis 2 (two 16-row tiles of M_2), plus 8 of padding: the
// host copy of the tile ranges k_tab_ktiles builds on the device (row k of
// M spans the free sets of the blocks holding k: blo..bhi, or its owner).
int fuse21_ldw(const Handle &h, int *maxnc) {
  const Axis &X = h.ax[2];
  const int n = X.n, ntiles = (n + 15) / 16;
  if (maxnc) *maxnc = 0;
  std::vector<int> lo(ntiles), hi(ntiles);
  for (int t = 0; t < ntiles; ++t) {
    int l = 1 << 30, u = 0;
    for (int k = 16 * t; k < std::min(n, 16 * t + 16); ++k) {
      int b0 = X.blo[k], b1 = X.bhi[k];
      if (h.combine == MFA_COMBINE_RAS) b0 = b1 = X.owner[k];
      l = std::min(l, X.blk[b0].F0);
      u = std::max(u, X.blk[b1].F1);
    }
    l &= ~7;
    lo[t] = l;
    hi[t] = l + 32 * ((u - l + 31) / 32);
    if (maxnc) *maxnc = std::max(*maxnc, (u - l + 31) / 32);
  }
  int w = 0;
  for (int t = 0; t < ntiles; t += kIT / 16) {
    int l = lo[t], u = hi[t];
    if (t + 1 < ntiles) {
      l = std::min(l, lo[t + 1]);
      u = std::max(u, hi[t + 1]);
    }
    w = std::max(w, u - l);
  }
  return w > 0 ? w + 8 : 0;
}

// workgroup LDS of the fused axis-2/axis-1 pass and the widest staged column
// range of phase 1 (two output tiles of M_2)
static size_t fused21_lds(const Axis &X1, int ldw) {
  return sizeof(__hip_bfloat16) * 2 * ((size_t)kIT * (X1.npad + 8) + 32 * (size_t)ldw);
}

bool mfma_fused21_ok(const Handle &h) {
  // phase 1 holds every 32-column K chunk of a tile's M_2 rows in registers:
  // at most kPre of them
  int maxnc = 0;
  const int ldw = fuse21_ldw(h, &maxnc);
  return h.ax[1].active && h.ax[2].active && h.ax[2].n >= 16 && ldw > 0 && maxnc <= kPre &&
         32 * ((ldw - 8) / 8) <= 512 && fused21_lds(h.ax[1], ldw) <= 64 * 1024 &&
         (int64_t)h.ax[0].n * nblk(h.ax[2].n, kIT) < (1ll << 31);
}

hipError_t launch_mfma_fused21(Handle &h, const float *in, float *out) {
  const Axis &X1 = h.ax[1], &X2 = h.ax[2];
  const int nr1 = (X1.n + 15) / 16 * 16, nr2 = (X2.n + 15) / 16 * 16;
  const __hip_bfloat16 *M1hi = reinterpret_cast<const __hip_bfloat16 *>(X1.d_Mb);
  const __hip_bfloat16 *M1lo = M1hi + (int64_t)nr1 * X1.npad;
  const __hip_bfloat16 *M2hi = reinterpret_cast<const __hip_bfloat16 *>(X2.d_Mb);
  const __hip_bfloat16 *M2lo = M2hi + (int64_t)nr2 * X2.npad;
  const int ldw = fuse21_ldw(h);
  const unsigned nb2 = nblk(X2.n, kIT);
  const int nch = (X1.n + 31) / 32;
#define MFA_F21(V, N)                                                                               \
  k_mfma_fused21<V, N><<<nb2 * (unsigned)h.ax[0].n, 256, fused21_lds(X1, ldw), h.stream>>>(         \
      in, out, X1.n, X2.n, X1.npad, X2.npad, M1hi, M1lo, X1.d_klo, X1.d_knc, M2hi, M2lo, X2.d_klo, \
      X2.d_knc, ldw, (int)nb2)
#define MFA_F21N(V)                      \
  switch (nch) {                         \
    case 4: MFA_F21(V, 4); break;        \
    case 6: MFA_F21(V, 6); break;        \
    case 8: MFA_F21(V, 8); break;        \
    case 12: MFA_F21(V, 12); break;      \
    case 16: MFA_F21(V, 16); break;      \
    default: MFA_F21(V, 0); break;       \
  }
  // 16-byte row loads need rows (and the array) 16-byte aligned
  if (X2.n % 4 == 0) {
    MFA_F21N(true)
  } else {
    MFA_F21N(false)
  }
#undef MFA_F21N
#undef MFA_F21
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
    // 16-byte row loads need rows 16-byte aligned
#define MFA_MC(M, V)                                                                             \
  k_mfma_contig<M, V><<<grid, threads, lds, h.stream>>>(in, out, h.P, n, nlines, X.npad, Mhi, Mlo, \
                                                        X.d_klo, X.d_knc, h.slots)
    const bool vec = n % 4 == 0;
    if (add) {
      if (vec) MFA_MC(1, true);
      else MFA_MC(1, false);
    } else {
      if (vec) MFA_MC(0, true);
      else MFA_MC(0, false);
    }
#undef MFA_MC
  } else {
    const int64_t outer = axis == 0 ? 1 : h.ax[0].n;
    const int64_t inner = axis == 0 ? (int64_t)h.ax[1].n * h.ax[2].n : h.ax[2].n;
    const dim3 grid(nblk(inner, kIT), (unsigned)outer);
    const size_t lds = mfma_lds(X.npad);
    if (add && axis == 0 && n <= 64 * kPT) {
      k_mfma_axis0_add<<<grid, 256, lds, h.stream>>>(in, h.P, n, inner, X.npad, Mhi, Mlo, X.d_klo,
                                                     X.d_knc, h.slots);
    } else if (add)
      k_mfma_strided<1><<<grid, 256, lds, h.stream>>>(in, out, h.P, n, inner, X.npad, Mhi, Mlo,
                                                      X.d_klo, X.d_knc, h.slots);
    else
      k_mfma_strided<0><<<grid, 256, lds, h.stream>>>(in, out, h.P, n, inner, X.npad, Mhi, Mlo,
                                                      X.d_klo, X.d_knc, h.slots);
  }
  return hipGetLastError();
}

}  // namespace mfa
