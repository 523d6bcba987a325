// Schwarz sweep kernels on the control grid.
//
//  k_resid  : g = c - (A_0 x A_1 x A_2) P, the local right-hand sides
//             N_F^T (Q - N P) of every subdomain at once (A_a = N_a^T N_a is
//             banded with half-width p).  One fused 3-D stencil: axis 2 and 1
//             from an LDS tile, axis 0 streamed through a register ring.
//  k_bsolve : the weighted additive-Schwarz correction along one axis,
//             out = sum_b w_b R_b^T (L_b L_b^T)^{-1} R_b in, by forward and
//             backward substitution with every subdomain's banded Cholesky
//             factor (the batched banded solves), one line per lane, the
//             1/n_s combine of overlapping segments done in LDS.
#include <cstdlib>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>
#include "mfa_internal.hpp"

namespace mfa {

namespace {

__device__ __forceinline__ void slot_max_c(unsigned long long *slots, int slot, double v) {
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
__device__ __forceinline__ void block_slot_max_c(unsigned long long *slots, int slot, double v) {
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

template <typename T>
__device__ __forceinline__ double to_d(T v) {
  return (double)v;
}
template <>
__device__ __forceinline__ double to_d<__hip_bfloat16>(__hip_bfloat16 v) {
  return (double)__bfloat162float(v);
}
template <typename T>
__device__ __forceinline__ T from_d(double v) {
  return (T)v;
}
template <>
__device__ __forceinline__ __hip_bfloat16 from_d<__hip_bfloat16>(double v) {
  return __float2bfloat16((float)v);
}

constexpr int kTZ = 64;   // z outputs per workgroup (one per lane)
constexpr int kTY = 16;   // y outputs per workgroup
constexpr int kRY = 2;    // y outputs per thread
constexpr int kRT = 512;  // threads per workgroup (kTY / kRY wavefronts)
// a buffer offset beyond every range the residual builds (ranges stay below
// 2^31 bytes, which the launcher checks)
constexpr unsigned kOOB = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer descriptor over `bytes` bytes from p (no stride, 32-bit data
// format): a load past the range returns zero and a store past it is
// dropped.  The residual takes its zero halo (cells outside the array,
// planes outside the array) and its discarded outputs (points past the
// array's edge, planes another chunk owns) from this range check instead
// of lane masks and branches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}
__device__ __forceinline__ double buf_ld64(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <typename TG>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double v);
template <>
__device__ __forceinline__ void buf_st<float>(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void buf_st<double>(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void buf_st<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, unsigned off,
                                                       double v) {
  __builtin_amdgcn_raw_buffer_store_b16(
      __builtin_bit_cast(unsigned short, __float2bfloat16((float)v)), r, (int)off, 0, 0);
}
// lane l's value of v, as a wave-uniform (scalar) value
__device__ __forceinline__ double lane_value(double v, int l) {
  const u32x2 b = __builtin_bit_cast(u32x2, v);
  u32x2 o;
  o.x = (unsigned)__builtin_amdgcn_readlane((int)b.x, l);
  o.y = (unsigned)__builtin_amdgcn_readlane((int)b.y, l);
  return __builtin_bit_cast(double, o);
}

// Coefficient tables Aa[k*(2P+1) + t] = A_a[k][k-P+t] (0 outside the matrix);
// an inactive axis (length 1) has the identity row.
template <int P, typename TG>
__global__ void __launch_bounds__(kRT, (P <= 4 ? 4 : 1)) k_resid(const double *__restrict__ Pc,
                                               const double *__restrict__ c, TG *__restrict__ g,
                                               const double *__restrict__ A0,
                                               const double *__restrict__ A1,
                                               const double *__restrict__ A2, int n0, int n1, int n2,
                                               int xchunk, unsigned long long *slots, SlotTurn turn) {
  constexpr int W = 2 * P + 1;
  constexpr int LY = kTY + 2 * P;
  constexpr int LZ = kTZ + 2 * P;
  constexpr int NE = (LY * LZ + kRT - 1) / kRT;   // tile elements per thread
  constexpr int NZR = (LY + 7) / 8;               // z-pass rows per wavefront
  // tile rows: the z pass reads rows up to 8 NZR - 1, and the flat stores of
  // the last element group run past LY LZ (rows beyond LY are never used)
  constexpr int TR = (8 * NZR > (NE * kRT + LZ - 1) / LZ) ? 8 * NZR : (NE * kRT + LZ - 1) / LZ;
  // double-buffered by plane parity (one barrier per plane, see below);
  // tile rows are unpadded (every access is contiguous across the lanes)
  __shared__ double tile[2][TR * LZ];
  __shared__ double tz[2][8 * NZR][kTZ + 1];
  const int tx = threadIdx.x & 63;
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wavefront index 0..7
  // Workgroups are dealt to the 8 XCDs round-robin in launch order.  Renumber
  // them (a bijection) so that each XCD takes a contiguous run of tiles with
  // y fastest, then z, then the x-chunk: tiles that share y and z halo rows
  // then stream the same planes at the same time through one L2.
  const unsigned gyz = gridDim.x * gridDim.y, G = gyz * gridDim.z;
  const unsigned L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned xcd = L % 8, per = G / 8, rem = G % 8;
  const unsigned lb = xcd * per + min(xcd, rem) + L / 8;
  const unsigned tyi = lb % gridDim.y, tzi = (lb / gridDim.y) % gridDim.x, txi = lb / gyz;
  const int z0 = tzi * kTZ, y0 = tyi * kTY, x0 = txi * xchunk;
  const int x1 = min(n0, x0 + xchunk);
  // slot bookkeeping (first workgroup): the previous sweep's max |correction|
  // into the history, then its slot set cleared for the next sweep; no other
  // kernel of this sweep touches that set
  if (turn.prev && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
    unsigned long long v = 0ull;
    if (threadIdx.x < kSlotCopies) v = turn.prev[kSlotMaxDP * kSlotCopies + threadIdx.x];
    if (turn.hist && threadIdx.x < 64) {
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
      }
      if (threadIdx.x == 0) turn.hist[turn.idx] = __longlong_as_double((long long)v);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNumSlots * kSlotCopies; e += kRT) turn.prev[e] = 0ull;
  }
  const int gz = z0 + tx;
  // Stencil rows of the points past the array's edge are zero, so that those
  // points' residuals are exactly 0 (their stores are dropped by the range
  // check and they do not reach the max |g| reduction).  This lane's axis-2
  // row stays in registers; the wavefront's two axis-1 rows are uniform and
  // loaded once.
  double az[W];
#pragma unroll
  for (int t = 0; t < W; ++t) az[t] = gz < n2 ? A2[(int64_t)gz * W + t] : 0.0;
  double ay[kRY][W];
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int gy = y0 + ty * kRY + r;
#pragma unroll
    for (int t = 0; t < W; ++t) ay[r][t] = gy < n1 ? A1[(int64_t)gy * W + t] : 0.0;
  }
  double ring[W][kRY];
#pragma unroll
  for (int t = 0; t < W; ++t)
#pragma unroll
    for (int r = 0; r < kRY; ++r) ring[t][r] = 0.0;
  double nres = 0.0;
  // Plane-invariant byte offsets: every thread's tile elements and output
  // points within a plane, kOOB where outside the array (the load then
  // returns 0, the store is dropped).
  const int64_t plane = (int64_t)n1 * n2;
  unsigned toff[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = threadIdx.x + kRT * i;
    const int yy = e / LZ, zz = e - yy * LZ;
    const int gy = y0 - P + yy, gzz = z0 - P + zz;
    const bool ok = e < LY * LZ && gy >= 0 && gy < n1 && gzz >= 0 && gzz < n2;
    toff[i] = ok ? (unsigned)(gy * n2 + gzz) * 8u : kOOB;
  }
  // right-hand side byte offsets of the thread's points; the output offset
  // is this shifted right by log2(8 / sizeof(TG)), which keeps kOOB past
  // the output's range
  unsigned coff[kRY];
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int gy = y0 + ty * kRY + r;
    coff[r] = (gy < n1 && gz < n2) ? (unsigned)(gy * n2 + gz) * 8u : kOOB;
  }
  constexpr int kGShift = sizeof(TG) == 8 ? 0 : sizeof(TG) == 4 ? 1 : 2;
  const int pbytes = (int)(plane * 8);
  // The tiles of the next two planes are in flight in registers while the
  // current plane is computed (software pipelining of the global loads, two
  // buffers, the loop unrolled by two); the plane count is rounded up to
  // even so that no branch separates a load from its wait (the extra plane
  // writes nothing).  Every global access is a buffer access, so the loop
  // issues no scalar memory loads: their completion count is shared with
  // LDS operations and would make every LDS wait a full wait.
  // One barrier per plane: the step of plane xi stores its tile into the
  // buffer of its parity, waits once, then runs the z pass of plane xi
  // (tile -> tz of that parity) and the y and x passes of plane xi - 1 (from
  // the other tz buffer, written before the barrier).  A buffer is rewritten
  // two steps after it was read, with a barrier in between.
  double preA[NE], preB[NE];
  auto gload = [&](double (&buf)[NE], int xi) {
    const bool in = xi >= 0 && xi < n0;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(Pc + (in ? xi : 0) * plane, in ? pbytes : 0);
#pragma unroll
    for (int i = 0; i < NE; ++i) buf[i] = buf_ld64(r, toff[i]);
  };
  const int xs = x0 - P, npl = (x1 + P - xs + 1) & ~1;
  // y pass of plane xo + P from tz[q] (ring of the last W planes' results),
  // then, for an owned plane xo, its x pass and the residual (zero stencil
  // row and right-hand side elsewhere, store dropped)
  auto yx = [&](int q, int xo, double a0v, const double (&cv)[kRY]) {
    {
      // the kRY rows of a thread share W - 1 of their W taps: one read each
      double tcol[W + kRY - 1];
#pragma unroll
      for (int t = 0; t < W + kRY - 1; ++t) tcol[t] = tz[q][ty * kRY + t][tx];
#pragma unroll
      for (int r = 0; r < kRY; ++r) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < W; ++t) s += ay[r][t] * tcol[r + t];
#pragma unroll
        for (int t = 0; t < W - 1; ++t) ring[t][r] = ring[t + 1][r];
        ring[W - 1][r] = s;
      }
    }
    const bool own = xo >= x0 && xo < x1;
    const __amdgpu_buffer_rsrc_t rg =
        buf_rsrc(g + (own ? xo : 0) * plane, own ? (int)(plane * sizeof(TG)) : 0);
    double axv[W];
#pragma unroll
    for (int t = 0; t < W; ++t) axv[t] = lane_value(a0v, t);
#pragma unroll
    for (int r = 0; r < kRY; ++r) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < W; ++t) s += axv[t] * ring[t][r];
      const double gv = cv[r] - s;
      buf_st<TG>(rg, coff[r] >> kGShift, gv);
      nres = fmax(nres, fabs(gv));
    }
  };
  // right-hand side and axis-0 stencil row of output plane xo (lane t < W
  // holds the row's t-th coefficient; zero for a plane this chunk does not own)
  auto rhs = [&](int xo, double &a0v, double (&cv)[kRY]) {
    const bool own = xo >= x0 && xo < x1;
    const __amdgpu_buffer_rsrc_t rc = buf_rsrc(c + (own ? xo : 0) * plane, own ? pbytes : 0);
#pragma unroll
    for (int r = 0; r < kRY; ++r) cv[r] = buf_ld64(rc, coff[r]);
    const __amdgpu_buffer_rsrc_t ra = buf_rsrc(A0, n0 * W * 8);
    a0v = buf_ld64(ra, own ? (unsigned)(xo * W + min(tx, W - 1)) * 8u : kOOB);
  };
  auto step = [&](double (&buf)[NE], int xi, int q) {
#pragma unroll
    for (int i = 0; i < NE; ++i) tile[q][threadIdx.x + kRT * i] = buf[i];
    // the right-hand side of the plane output in this step, requested after
    // the wait for the tile (loads return in order) and before the tile two
    // planes ahead, so that neither wait covers the other
    double a0v, cv[kRY];
    rhs(xi - 1 - P, a0v, cv);
    __syncthreads();
    // past the chunk's last plane the prefetch re-reads that plane (cache
    // hits, never used) instead of the next chunk's planes
    gload(buf, min(xi + 2, x1 + P - 1));
    // z pass: a wavefront's rows ty, ty + 8, ... as independent chains
    // (rows past LY are computed from unused tile rows and never read)
#pragma unroll
    for (int k = 0; k < NZR; ++k) {
      const double *tr = &tile[q][(ty + 8 * k) * LZ + tx];
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < W; ++t) s += az[t] * tr[t];
      tz[q][ty + 8 * k][tx] = s;
    }
    if (xi > xs) yx(q ^ 1, xi - 1 - P, a0v, cv);
  };
  gload(preA, xs);
  // keep A's loads ahead of B's: the waits count loads in issue order
  asm volatile("" ::: "memory");
  gload(preB, xs + 1);
  for (int xi = xs; xi < xs + npl; xi += 2) {
    step(preA, xi, 0);
    step(preB, xi + 1, 1);
  }
  {
    // the last plane's y and x passes (its z pass went to tz[1]: npl is even)
    double a0v, cv[kRY];
    rhs(xs + npl - 1 - P, a0v, cv);
    __syncthreads();
    yx(1, xs + npl - 1 - P, a0v, cv);
  }
  block_slot_max_c(slots, kSlotNres, nres);
}

// Line geometry of an axis pass on an (n0, n1, n2) array: `nlines` lines of
// length `len`, element j of line l at base(l) + j*stride.
struct LineGeom {
  int axis;   // 0, 1, 2
  int n0, n1, n2;
};

__device__ __forceinline__ int64_t line_base(const LineGeom &G, int64_t l) {
  if (G.axis == 0) return l;                                    // l = y*n2 + z
  if (G.axis == 1) return (l / G.n2) * (int64_t)G.n1 * G.n2 + (l % G.n2);  // l = x*n2 + z
  return l * G.n2;                                              // l = x*n1 + y
}

__device__ __forceinline__ int64_t line_stride(const LineGeom &G) {
  return G.axis == 0 ? (int64_t)G.n1 * G.n2 : (G.axis == 1 ? G.n2 : 1);
}

// Weighted additive-Schwarz correction along one axis, 64 lines per
// workgroup (one per lane).  For every subdomain b of the axis, in order:
//  1. the factor L_b (band, (P+1) x F) and its reciprocal pivots go to LDS;
//  2. the segment F_b of each line goes to LDS (coalesced: lanes over lines
//     for axes 0/1; lanes over the contiguous segment for axis 2);
//  3. forward then backward substitution, the last P values of the
//     recurrence kept in registers;
//  4. positions [F0_b, F0_{b+1}) are final: the part shared with the previous
//     segment sums the two ping-pong buffers with weight 1/n_s (AVG), or takes
//     the owner's value (RAS).  Axis 2 stages them in LDS (in the buffer of
//     the previous segment, compacted in place) and stores them coalesced.
// MODE 0 stores the correction, MODE 1 adds it to `pc` (the control points)
// and reduces max |correction|.
template <typename TI, typename TO, typename TC, int MODE, int P>
__global__ void __launch_bounds__(64) k_bsolve(const TI *__restrict__ in, TO *__restrict__ out,
                                               double *__restrict__ pc, LineGeom G, int64_t nlines,
                                               int B, const int *__restrict__ blk,
                                               const int *__restrict__ choff,
                                               const double *__restrict__ chol,
                                               const int *__restrict__ foff,
                                               const double *__restrict__ rdiag,
                                               const int *__restrict__ ns, int combine, int flen,
                                               unsigned long long *slots) {
  constexpr int LS = 65;   // row stride of the line buffers (odd: no bank conflicts)
  extern __shared__ double smem_d[];
  double *fac = smem_d;                             // [(P+1) * flen]
  double *rdl = smem_d + (P + 1) * flen;            // [flen]
  TC *buf = reinterpret_cast<TC *>(smem_d + (P + 2) * flen);   // [2][flen][LS]
  const int lane = threadIdx.x;
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const int64_t l = l0 + lane;
  const bool valid = l < nlines;
  const int64_t stride = line_stride(G);
  const int64_t base = valid ? line_base(G, l) : 0;
  const bool inner = G.axis == 2;
  const int nin = (int)min<int64_t>(64, nlines - l0);   // lines in this workgroup
  double dmax = 0.0;
  int prevF0 = 0, prevF1 = 0;
  for (int b = 0; b < B; ++b) {
    TC *cur = buf + (size_t)(b & 1) * flen * LS;
    TC *prv = buf + (size_t)((b + 1) & 1) * flen * LS;
    const int F0 = blk[8 * b + 2], F1 = blk[8 * b + 3], F = F1 - F0;
    const int c0 = blk[8 * b + 0], c1 = blk[8 * b + 1];
    __syncthreads();   // previous segment's readers of fac/rdl/buffers are done
    {
      const double *L = chol + choff[b];
      for (int e = lane; e < (P + 1) * F; e += 64) fac[e] = L[e];
      const double *rd = rdiag + foff[b];
      for (int e = lane; e < F; e += 64) rdl[e] = rd[e];
    }
    if (inner) {
      for (int e = lane; e < nin * F; e += 64) {
        const int li = e / F, j = e - li * F;
        cur[j * LS + li] = (TC)to_d(in[(l0 + li) * G.n2 + F0 + j]);
      }
    } else if (valid) {
      for (int j = 0; j < F; ++j) cur[j * LS + lane] = (TC)to_d(in[base + (int64_t)(F0 + j) * stride]);
    }
    __syncthreads();
    // forward: L y = s;  w[t] = y_{j-1-t}.  The next step's input and
    // coefficients are read ahead so LDS latency overlaps the FMA chain.
    {
      TC w[P];
#pragma unroll
      for (int t = 0; t < P; ++t) w[t] = (TC)0;
      TC sn = cur[lane];
      TC cn[P];
#pragma unroll
      for (int t = 1; t <= P; ++t) cn[t - 1] = (TC)fac[t * F - t];
      TC rn = (TC)rdl[0];
      for (int j = 0; j < F; ++j) {
        TC s = sn, r = rn;
        TC cc[P];
#pragma unroll
        for (int t = 0; t < P; ++t) cc[t] = cn[t];
        if (j + 1 < F) {
          sn = cur[(j + 1) * LS + lane];
#pragma unroll
          for (int t = 1; t <= P; ++t) cn[t - 1] = (TC)fac[t * F + (j + 1 - t)];
          rn = (TC)rdl[j + 1];
        }
#pragma unroll
        for (int t = 1; t <= P; ++t) s -= cc[t - 1] * w[t - 1];
        const TC y = s * r;
#pragma unroll
        for (int t = P - 1; t > 0; --t) w[t] = w[t - 1];
        w[0] = y;
        cur[j * LS + lane] = y;
      }
    }
    // backward: L^T x = y;  w[t] = x_{j+1+t}
    {
      TC w[P];
#pragma unroll
      for (int t = 0; t < P; ++t) w[t] = (TC)0;
      TC sn = cur[(F - 1) * LS + lane];
      TC cn[P];
#pragma unroll
      for (int t = 1; t <= P; ++t) cn[t - 1] = (TC)fac[t * F + F - 1];
      TC rn = (TC)rdl[F - 1];
      for (int j = F - 1; j >= 0; --j) {
        TC s = sn, r = rn;
        TC cc[P];
#pragma unroll
        for (int t = 0; t < P; ++t) cc[t] = cn[t];
        if (j > 0) {
          sn = cur[(j - 1) * LS + lane];
#pragma unroll
          for (int t = 1; t <= P; ++t) cn[t - 1] = (TC)fac[t * F + j - 1];
          rn = (TC)rdl[j - 1];
        }
#pragma unroll
        for (int t = 1; t <= P; ++t) s -= cc[t - 1] * w[t - 1];
        const TC x = s * r;
#pragma unroll
        for (int t = P - 1; t > 0; --t) w[t] = w[t - 1];
        w[0] = x;
        cur[j * LS + lane] = x;
      }
    }
    // combine the final positions of this segment
    const int whi = b + 1 < B ? blk[8 * (b + 1) + 2] : F1;
    const int pc0 = b > 0 ? blk[8 * (b - 1) + 0] : 0, pc1 = b > 0 ? blk[8 * (b - 1) + 1] : 0;
    for (int k = F0; k < whi; ++k) {
      double v;
      if (combine == MFA_COMBINE_RAS) {
        if (k >= c0 && k < c1) v = (double)cur[(k - F0) * LS + lane];
        else if (b > 0 && k < prevF1 && k >= pc0 && k < pc1) v = (double)prv[(k - prevF0) * LS + lane];
        else v = 0.0;
      } else {
        v = (double)cur[(k - F0) * LS + lane];
        if (b > 0 && k < prevF1) v += (double)prv[(k - prevF0) * LS + lane];
        v /= (double)ns[k];
      }
      if (MODE == 1) dmax = fmax(dmax, valid ? fabs(v) : 0.0);
      if (inner) {
        // in place: slot k-F0 <= k-prevF0, already read for this and earlier k
        prv[(k - F0) * LS + lane] = (TC)v;
      } else if (valid) {
        const int64_t o = base + (int64_t)k * stride;
        if (MODE == 0) out[o] = from_d<TO>(v);
        else pc[o] = pc[o] + v;
      }
    }
    if (inner) {
      __syncthreads();
      const int W = whi - F0;
      for (int e = lane; e < nin * W; e += 64) {
        const int li = e / W, j = e - li * W;
        const int64_t o = (l0 + li) * G.n2 + F0 + j;
        const double v = (double)prv[j * LS + li];
        if (MODE == 0) out[o] = from_d<TO>(v);
        else pc[o] = pc[o] + v;
      }
    }
    prevF0 = F0;
    prevF1 = F1;
  }
  if (MODE == 1) slot_max_c(slots, kSlotMaxDP, dmax);
}

// Segment-parallel variant: one lane per (line, subdomain segment).  A
// workgroup holds 64 lines x B segments (B <= 16), lane = b*64 + line, so a
// wavefront is one segment of 64 consecutive lines (coalesced on axes 0/1).
// The segment (length F <= MAXF) lives in registers: the substitutions are
// fully unrolled; the factor entries are wavefront-uniform (scalar loads).
// Each segment publishes its tail (the positions it shares with the next
// segment) in LDS; after one barrier every segment writes the positions
// [F0_b, F0_{b+1}), adding the left neighbour's tail on the shared part with
// weight 1/n_s (AVG) or taking the owner's value (RAS).
template <typename TI, typename TO, typename TC, int MODE, int MAXF>
__global__ void __launch_bounds__(MAXF >= 64 ? 256 : 1024) k_bsolve_seg(const TI *__restrict__ in,
                                                                          TO *__restrict__ out,
                                                     double *__restrict__ pc, LineGeom G,
                                                     int64_t nlines, int p, int B,
                                                     const int *__restrict__ blk,
                                                     const int *__restrict__ choff,
                                                     const double *__restrict__ chol,
                                                     const int *__restrict__ foff,
                                                     const double *__restrict__ rdiag,
                                                     const int *__restrict__ ns, int combine, int ov,
                                                     unsigned long long *slots) {
  extern __shared__ double smem_t[];
  TC *tails = reinterpret_cast<TC *>(smem_t);   // [B][64][ov]
  const int li = threadIdx.x & 63;
  const int b = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t l = (int64_t)blockIdx.x * 64 + li;
  const bool valid = l < nlines;
  const int64_t stride = line_stride(G);
  const int64_t base = valid ? line_base(G, l) : 0;
  const int F0 = blk[8 * b + 2], F1 = blk[8 * b + 3], F = F1 - F0;
  const int c0 = blk[8 * b + 0], c1 = blk[8 * b + 1];
  const int F0n = b + 1 < B ? blk[8 * (b + 1) + 2] : F1;
  const double *L = chol + choff[b];
  const double *rd = rdiag + foff[b];
  TC x[MAXF];
#pragma unroll
  for (int j = 0; j < MAXF; ++j)
    if (j < F) x[j] = valid ? (TC)to_d(in[base + (int64_t)(F0 + j) * stride]) : (TC)0;
  // forward: L y = s
#pragma unroll
  for (int j = 0; j < MAXF; ++j) {
    if (j < F) {
      TC s = x[j];
#pragma unroll
      for (int t = 1; t <= kMaxP; ++t)
        if (t <= j && t <= p) s -= (TC)L[t * F + (j - t)] * x[j - t];
      x[j] = s * (TC)rd[j];
    }
  }
  // backward: L^T x = y
#pragma unroll
  for (int j = MAXF - 1; j >= 0; --j) {
    if (j < F) {
      TC s = x[j];
#pragma unroll
      for (int t = 1; t <= kMaxP; ++t)
        if (j + t < MAXF && t <= p && j + t < F) s -= (TC)L[t * F + j] * x[j + t];
      x[j] = s * (TC)rd[j];
    }
  }
  // publish the tail shared with the next segment
  TC *mytail = tails + ((size_t)b * 64 + li) * ov;
#pragma unroll
  for (int j = 0; j < MAXF; ++j)
    if (j < F && F0 + j >= F0n) mytail[F0 + j - F0n] = x[j];
  __syncthreads();
  const TC *lefttail = b > 0 ? tails + ((size_t)(b - 1) * 64 + li) * ov : nullptr;
  const int F1p = b > 0 ? blk[8 * (b - 1) + 3] : 0;
  const int c0p = b > 0 ? blk[8 * (b - 1) + 0] : 0, c1p = b > 0 ? blk[8 * (b - 1) + 1] : 0;
  double dmax = 0.0;
#pragma unroll
  for (int j = 0; j < MAXF; ++j) {
    const int k = F0 + j;
    if (j < F && k < F0n) {
      double v;
      const bool shared_left = b > 0 && k < F1p;
      if (combine == MFA_COMBINE_RAS) {
        if (k >= c0 && k < c1) v = (double)x[j];
        else if (shared_left && k >= c0p && k < c1p) v = (double)lefttail[k - F0];
        else v = 0.0;
      } else {
        v = (double)x[j];
        if (shared_left) v += (double)lefttail[k - F0];
        v /= (double)ns[k];
      }
      if (valid) {
        const int64_t o = base + (int64_t)k * stride;
        if (MODE == 0) {
          out[o] = from_d<TO>(v);
        } else {
          pc[o] = pc[o] + v;
          dmax = fmax(dmax, fabs(v));
        }
      }
    }
  }
  if (MODE == 1) block_slot_max_c(slots, kSlotMaxDP, dmax);
}

// The residual at P = 0 (the first sweep of a cold start): the stencil of
// zeros is zero, so g = c exactly, and max |g| goes to the residual slot as
// k_resid would put it.  Four values per thread and trip, 16-byte accesses
// (c and g start on 16-byte boundaries: workspace arrays).
template <typename TG>
__device__ __forceinline__ void store4(TG *g, double a, double b, double c, double d);
template <>
__device__ __forceinline__ void store4<float>(float *g, double a, double b, double c, double d) {
  *reinterpret_cast<float4 *>(g) = float4{(float)a, (float)b, (float)c, (float)d};
}
template <>
__device__ __forceinline__ void store4<double>(double *g, double a, double b, double c, double d) {
  reinterpret_cast<double2 *>(g)[0] = double2{a, b};
  reinterpret_cast<double2 *>(g)[1] = double2{c, d};
}
template <typename TG>
__global__ void __launch_bounds__(256) k_resid_zero(const double *__restrict__ c, TG *__restrict__ g,
                                                   int64_t n, unsigned long long *slots) {
  double nres = 0.0;
  const int64_t n4 = n / 4, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < n4; i += stride) {
    const double2 a = reinterpret_cast<const double2 *>(c)[2 * i];
    const double2 b = reinterpret_cast<const double2 *>(c)[2 * i + 1];
    store4<TG>(g + 4 * i, a.x, a.y, b.x, b.y);
    nres = fmax(nres, fmax(fmax(fabs(a.x), fabs(a.y)), fmax(fabs(b.x), fabs(b.y))));
  }
  for (int64_t i = 4 * n4 + t0; i < n; i += stride) {
    const double v = c[i];
    g[i] = from_d<TG>(v);
    nres = fmax(nres, fabs(v));
  }
  block_slot_max_c(slots, kSlotNres, nres);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// x-chunk of the residual stencil for at most `target` workgroups: the
// number of chunks is chosen first (the most that keeps byz x chunks within
// the target, each chunk at least 4 planes) and the planes are then spread
// evenly over them.  Each chunk re-reads 2p halo planes; a target of twice
// the CU count lets two workgroups share every CU without a third one
// lengthening some CU's queue.
inline int resid_xchunk(int n0, int byz, int target) {
  const int nch = std::max(1, std::min(target / byz, n0 / 4));
  return (n0 + nch - 1) / nch;
}

// Autotuned x-chunk per shape.  The residual is idempotent (it reads P and c
// and writes g), and every output's arithmetic is the same whatever the
// chunking, so on the first launch for a large shape each candidate runs on
// the live arrays and is timed with events; the fastest is kept for the life
// of the process.  Small shapes take the heuristic choice untimed.
struct ResidKey {
  int n0, n1, n2, p, tg;
  bool operator<(const ResidKey &o) const {
    return std::tie(n0, n1, n2, p, tg) < std::tie(o.n0, o.n1, o.n2, o.p, o.tg);
  }
};
std::mutex g_resid_mu;
std::map<ResidKey, int> g_resid_chunk;
constexpr int64_t kTuneMinCtrl = 1 << 20;

template <int P, typename TG>
hipError_t launch_resid_p(hipStream_t st, const double *Pc, const double *c, TG *g, const double *A0,
                          const double *A1, const double *A2, int n0, int n1, int n2,
                          unsigned long long *slots, const SlotTurn &turn, bool may_tune) {
  // the kernel addresses a plane (and the axis-0 table) through buffer
  // ranges of fewer than 2^31 bytes
  if ((int64_t)n1 * n2 * 8 > INT32_MAX || (int64_t)n0 * (2 * P + 1) * 8 > INT32_MAX)
    return hipErrorInvalidValue;
  const int byz = (int)(nblk(n2, kTZ) * nblk(n1, kTY));
  const ResidKey key{n0, n1, n2, P, (int)sizeof(TG)};
  int xchunk = 0;
  {
    std::lock_guard<std::mutex> lk(g_resid_mu);
    auto it = g_resid_chunk.find(key);
    if (it != g_resid_chunk.end()) xchunk = it->second;
  }
  // the tuner's timing launches skip the slot bookkeeping (recording the
  // history is not idempotent); the sweep's own launch does it
  auto launch = [&](int xc, const SlotTurn &tn) {
    const dim3 grid(nblk(n2, kTZ), nblk(n1, kTY), nblk(n0, xc));
    k_resid<P, TG><<<grid, kRT, 0, st>>>(Pc, c, g, A0, A1, A2, n0, n1, n2, xc, slots, tn);
    return hipGetLastError();
  };
  // MFA_RESID_XCHUNK=n (n > 0) pins the chunk for every shape and skips the
  // tuner (read on every launch): a profiler's per-dispatch overhead can
  // change the tuner's choice, and counters must be taken on the
  // configuration that is timed
  if (const char *pin = getenv("MFA_RESID_XCHUNK")) {
    const int v = atoi(pin);
    if (v > 0) xchunk = std::min(v, n0);
  }
  if (xchunk == 0) {
    // default: at most 512 workgroups, two per CU (on 256 x 256 x 192
    // control points: 10 chunks of 26 planes, 480 workgroups, 8% less
    // time than 5 chunks of 48 planes plus one of 16, and 25% less than 6
    // even chunks of 43 planes, which put two long chunks on 32 CUs),
    // unless that leaves chunks shorter than 4p planes, whose 2p halo
    // planes would cost more than the second workgroup per CU gains: then
    // at most 256 (128^3, p = 3: 8-plane chunks 31-33 us, 4-plane chunks
    // 34 us); 768 for small shapes
    const int64_t nctrl = (int64_t)n0 * n1 * n2;
    int xdef = resid_xchunk(n0, byz, nctrl >= kTuneMinCtrl ? 512 : 768);
    if (nctrl >= kTuneMinCtrl && xdef < 4 * P) xdef = resid_xchunk(n0, byz, 256);
    xchunk = xdef;
    if (!may_tune) return launch(xdef, turn);   // untimed, not cached
    if (nctrl >= kTuneMinCtrl) {
      std::vector<int> cand{xdef};
      for (int target : {256, 384, 512, 768, 1024, 1536}) {
        const int xc = resid_xchunk(n0, byz, target);
        if (std::find(cand.begin(), cand.end(), xc) == cand.end()) cand.push_back(xc);
      }
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess) return hipErrorOutOfMemory;
      if (hipEventCreate(&e1) != hipSuccess) return hipErrorOutOfMemory;
      // each candidate timed three times (fastest kept); the default stays
      // unless a candidate is at least 10% faster, so that timing noise
      // (or a profiler's overhead) cannot flip the choice
      std::vector<float> tmin(cand.size(), 1e30f);
      hipError_t err = launch(cand[0], SlotTurn{});   // warm-up
      for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
        for (size_t i = 0; i < cand.size() && err == hipSuccess; ++i) {
          float ms = 0.f;
          hipEventRecord(e0, st);
          err = launch(cand[i], SlotTurn{});
          hipEventRecord(e1, st);
          if (err == hipSuccess) err = hipEventSynchronize(e1);
          if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
          if (err == hipSuccess) tmin[i] = std::min(tmin[i], ms);
        }
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      if (err != hipSuccess) return err;
      const size_t ib = std::min_element(tmin.begin(), tmin.end()) - tmin.begin();
      const size_t id = std::find(cand.begin(), cand.end(), xdef) - cand.begin();
      xchunk = tmin[ib] < 0.9f * tmin[id] ? cand[ib] : xdef;
    }
    std::lock_guard<std::mutex> lk(g_resid_mu);
    g_resid_chunk[key] = xchunk;
  }
  return launch(xchunk, turn);
}

}  // namespace

template <typename TG>
hipError_t launch_resid(hipStream_t st, int p, const double *Pc, const double *c, TG *g,
                        const double *A0, const double *A1, const double *A2, int n0, int n1, int n2,
                        unsigned long long *slots, const SlotTurn &turn, bool may_tune) {
  switch (p) {
#define MFA_RESID_CASE(PP) \
  case PP:                 \
    return launch_resid_p<PP, TG>(st, Pc, c, g, A0, A1, A2, n0, n1, n2, slots, turn, may_tune);
    MFA_RESID_CASE(1)
    MFA_RESID_CASE(2)
    MFA_RESID_CASE(3)
    MFA_RESID_CASE(4)
    MFA_RESID_CASE(5)
    MFA_RESID_CASE(6)
    MFA_RESID_CASE(7)
    MFA_RESID_CASE(8)
#undef MFA_RESID_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TI, typename TO, typename TC, int MAXF>
hipError_t launch_bsolve_seg(hipStream_t st, const TI *in, TO *out, double *pc, LineGeom G,
                             int64_t nlines, int p, const Axis &X, int combine, int ov,
                             unsigned long long *slots) {
  const unsigned grid = nblk(nlines, 64);
  const size_t lds = sizeof(TC) * (size_t)X.B * 64 * std::max(ov, 1);
  if (pc)
    k_bsolve_seg<TI, TO, TC, 1, MAXF><<<grid, 64 * X.B, lds, st>>>(
        in, out, pc, G, nlines, p, X.B, X.d_blk, X.d_choff, X.d_chol, X.d_foff, X.d_rdiag, X.d_ns,
        combine, std::max(ov, 1), slots);
  else
    k_bsolve_seg<TI, TO, TC, 0, MAXF><<<grid, 64 * X.B, lds, st>>>(
        in, out, pc, G, nlines, p, X.B, X.d_blk, X.d_choff, X.d_chol, X.d_foff, X.d_rdiag, X.d_ns,
        combine, std::max(ov, 1), slots);
  return hipGetLastError();
}

// segment-parallel banded solves (a wavefront per subdomain, segments held
// in registers): up to 16 subdomains per axis with segments of at most 48
// control points, up to 4 with segments of at most 64 (the wide variant runs
// 256-thread workgroups so its segments fit the registers)
bool bsolve_seg_ok(const Axis &X) { return (X.B <= 16 && X.Fmax <= 48) || (X.B <= 4 && X.Fmax <= 64); }

template <typename TI, typename TO, typename TC>
hipError_t launch_bsolve(hipStream_t st, const TI *in, TO *out, double *pc, int axis, int n0, int n1,
                         int n2, int p, const Axis &X, int combine, unsigned long long *slots) {
  LineGeom G{axis, n0, n1, n2};
  const int64_t len = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
  const int64_t nlines = (int64_t)n0 * n1 * n2 / len;
  if (bsolve_seg_ok(X)) {
    int ov = 0;
    for (int b = 0; b + 1 < X.B; ++b) ov = std::max(ov, X.blk[b].F1 - X.blk[b + 1].F0);
    if (X.Fmax <= 16) return launch_bsolve_seg<TI, TO, TC, 16>(st, in, out, pc, G, nlines, p, X, combine, ov, slots);
    if (X.Fmax <= 32) return launch_bsolve_seg<TI, TO, TC, 32>(st, in, out, pc, G, nlines, p, X, combine, ov, slots);
    if (X.Fmax <= 48) return launch_bsolve_seg<TI, TO, TC, 48>(st, in, out, pc, G, nlines, p, X, combine, ov, slots);
    return launch_bsolve_seg<TI, TO, TC, 64>(st, in, out, pc, G, nlines, p, X, combine, ov, slots);
  }
  const int flen = (int)X.Fmax;
  const size_t lds = bsolve_lds(flen, p, sizeof(TC));
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const unsigned grid = nblk(nlines, 64);
  switch (p * 2 + (pc ? 1 : 0)) {
#define MFA_BS_CASE(PP)                                                                              \
  case 2 * PP:                                                                                       \
    k_bsolve<TI, TO, TC, 0, PP><<<grid, 64, lds, st>>>(in, out, pc, G, nlines, X.B, X.d_blk,         \
                                                       X.d_choff, X.d_chol, X.d_foff, X.d_rdiag,     \
                                                       X.d_ns, combine, flen, slots);                \
    break;                                                                                           \
  case 2 * PP + 1:                                                                                   \
    k_bsolve<TI, TO, TC, 1, PP><<<grid, 64, lds, st>>>(in, out, pc, G, nlines, X.B, X.d_blk,         \
                                                       X.d_choff, X.d_chol, X.d_foff, X.d_rdiag,     \
                                                       X.d_ns, combine, flen, slots);                \
    break;
    MFA_BS_CASE(1)
    MFA_BS_CASE(2)
    MFA_BS_CASE(3)
    MFA_BS_CASE(4)
    MFA_BS_CASE(5)
    MFA_BS_CASE(6)
    MFA_BS_CASE(7)
    MFA_BS_CASE(8)
#undef MFA_BS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TG>
hipError_t launch_resid_zero(hipStream_t st, const double *c, TG *g, int64_t n, unsigned long long *slots) {
  if (n <= 0) return hipSuccess;
  // four workgroups per CU: every wavefront ends with one atomic max on the
  // slot's copies, so more workgroups only queue more atomics at L2
  const unsigned grid = (unsigned)std::min<int64_t>(nblk((n + 3) / 4, 256), 1024);
  k_resid_zero<TG><<<grid, 256, 0, st>>>(c, g, n, slots);
  return hipGetLastError();
}
template hipError_t launch_resid_zero<double>(hipStream_t, const double *, double *, int64_t,
                                              unsigned long long *);
template hipError_t launch_resid_zero<float>(hipStream_t, const double *, float *, int64_t,
                                             unsigned long long *);

template hipError_t launch_resid<double>(hipStream_t, int, const double *, const double *, double *,
                                         const double *, const double *, const double *, int, int, int,
                                         unsigned long long *, const SlotTurn &, bool);
template hipError_t launch_resid<float>(hipStream_t, int, const double *, const double *, float *,
                                        const double *, const double *, const double *, int, int, int,
                                        unsigned long long *, const SlotTurn &, bool);
template hipError_t launch_resid<__hip_bfloat16>(hipStream_t, int, const double *, const double *,
                                                 __hip_bfloat16 *, const double *, const double *,
                                                 const double *, int, int, int, unsigned long long *,
                                                 const SlotTurn &, bool);
template hipError_t launch_bsolve<double, double, double>(hipStream_t, const double *, double *,
                                                          double *, int, int, int, int, int,
                                                          const Axis &, int, unsigned long long *);
template hipError_t launch_bsolve<float, float, float>(hipStream_t, const float *, float *, double *,
                                                       int, int, int, int, int, const Axis &, int,
                                                       unsigned long long *);

}  // namespace mfa
