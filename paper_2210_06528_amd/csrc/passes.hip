// Generic axis pass: apply a row-sparse operator along one axis of a 3-D
// array (the building block of every tensor-product contraction here), with
// an epilogue that stores, forms a residual, accumulates into the control
// points or only reduces max |value| into a slot.
#include "mfa_internal.hpp"

namespace mfa {

namespace {

__device__ __forceinline__ void slot_max(unsigned long long *slots, int slot, double v) {
  const unsigned copy =
      (blockIdx.x * 7u + blockIdx.y * 131u + blockIdx.z * 1031u + (threadIdx.x >> 6)) % kSlotCopies;
  atomicMax(slots + (size_t)slot * kSlotCopies + copy, (unsigned long long)__double_as_longlong(v));
}

// Wavefront max of v (non-negative) into slots[slot]; lanes may name
// different slots: one shuffle reduction and one atomic per distinct slot.
__device__ __forceinline__ void wave_slot_max(unsigned long long *slots, int slot, double v) {
  unsigned long long todo = __ballot(1);
  const int lane = __lane_id();
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int s = __shfl(slot, leader, 64);
    const bool mine = slot == s;
    double x = mine ? v : 0.0;
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    if (lane == leader) slot_max(slots, s, x);
    todo &= ~__ballot(mine);
  }
}

// Wavefront reduction of a data-residual value d into rs: max |d| (atomic max
// on the bit pattern) into copies [0, kSlotCopies), sum d^2 (atomic add) into
// copies [kSlotCopies, 2 kSlotCopies).
__device__ __forceinline__ void wave_res(unsigned long long *rs, double d) {
  double mx = fabs(d), sq = d * d;
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    sq += __shfl_xor(sq, off, 64);
  }
  if (__lane_id() == 0) {
    const unsigned copy =
        (blockIdx.x * 7u + blockIdx.y * 131u + blockIdx.z * 1031u + (threadIdx.x >> 6)) % kSlotCopies;
    atomicMax(rs + copy, (unsigned long long)__double_as_longlong(mx));
    atomicAdd(reinterpret_cast<double *>(rs + kSlotCopies + copy), sq);
  }
}

// One thread per output element; grid (ceil(o2/bs), o1, o0).  When the
// operator acts on axis 0 or 1 the row is uniform over the workgroup (table
// loads are scalar); on axis 2 each lane has its own row.
template <typename Tin, typename Tout, int EPI>
__global__ void __launch_bounds__(256) k_pass(const Tin *__restrict__ in, Tout *__restrict__ out,
                                              const double *__restrict__ sub, int o0, int o1, int o2,
                                              int ax, int rin, Ell op, unsigned long long *slots,
                                              int slot_base, const int *__restrict__ gid, int gaxis) {
  const int x2 = blockIdx.x * blockDim.x + threadIdx.x;
  const int x1 = blockIdx.y, x0 = blockIdx.z;
  const bool valid = x2 < o2;
  double acc = 0.0;
  int slot = slot_base;
  if (valid) {
    const int row = ax == 0 ? x0 : (ax == 1 ? x1 : x2);
    if (EPI == EPI_MAXABS && gid != nullptr) slot = slot_base + gid[gaxis == 0 ? x0 : (gaxis == 1 ? x1 : x2)];
    const int *cl = op.col + (int64_t)row * op.L;
    const double *vl = op.val + (int64_t)row * op.L;
    const int ln = op.len[row];
    if (ax == 0) {
      const int64_t plane = (int64_t)o1 * o2;
      const Tin *src = in + (int64_t)x1 * o2 + x2;
      for (int q = 0; q < ln; ++q) acc += vl[q] * (double)src[(int64_t)cl[q] * plane];
    } else if (ax == 1) {
      const Tin *src = in + (int64_t)x0 * rin * o2 + x2;
      for (int q = 0; q < ln; ++q) acc += vl[q] * (double)src[(int64_t)cl[q] * o2];
    } else {
      const Tin *src = in + ((int64_t)x0 * o1 + x1) * rin;
      for (int q = 0; q < ln; ++q) acc += vl[q] * (double)src[cl[q]];
    }
    const int64_t idx = ((int64_t)x0 * o1 + x1) * o2 + x2;
    if (EPI == EPI_STORE || EPI == EPI_STOREMAX) {
      out[idx] = (Tout)acc;
    } else if (EPI == EPI_SUBFROM) {
      acc = sub[idx] - acc;
      out[idx] = (Tout)acc;
    } else if (EPI == EPI_ADDTO) {
      out[idx] = (Tout)((double)out[idx] + acc);
    } else if (EPI == EPI_RESID32) {
      acc = (double)reinterpret_cast<const float *>(sub)[idx] - acc;
    } else if (EPI == EPI_RESID64) {
      acc = sub[idx] - acc;
    }
  }
  if (EPI == EPI_RESID32 || EPI == EPI_RESID64)
    wave_res(slots, valid ? acc : 0.0);
  else if (EPI != EPI_STORE)
    wave_slot_max(slots, slot, valid ? fabs(acc) : 0.0);
}

// point residual on the segmented data boxes: r = Q(gathered) - r
template <typename TQ>
__global__ void __launch_bounds__(256) k_box_resid(const TQ *__restrict__ q, int q1, int q2,
                                                   double *__restrict__ r, int r0, int r1, int r2,
                                                   const int *__restrict__ qm0,
                                                   const int *__restrict__ qm1,
                                                   const int *__restrict__ qm2) {
  const int x2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (x2 >= r2) return;
  const int x1 = blockIdx.y, x0 = blockIdx.z;
  const int i0 = qm0 ? qm0[x0] : 0, i1 = qm1 ? qm1[x1] : 0, i2 = qm2 ? qm2[x2] : 0;
  const int64_t ri = ((int64_t)x0 * r1 + x1) * r2 + x2;
  r[ri] = (double)q[((int64_t)i0 * q1 + i1) * q2 + i2] - r[ri];
}

__global__ void k_fill(double *x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// One wavefront per block; block 0 reads the kSlotCopies copies of slot
// kSlotMaxDP of `from` (max over the copies) before any clearing.
__global__ void k_zero_slots(unsigned long long *s, int n, double *hist, int idx,
                             const unsigned long long *from) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (hist && blockIdx.x == 0) {
    unsigned long long v = threadIdx.x < kSlotCopies ? from[kSlotMaxDP * kSlotCopies + threadIdx.x] : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    if (threadIdx.x == 0) hist[idx] = __longlong_as_double((long long)v);
  }
  if (i < n) s[i] = 0ull;
}

// out[s] = the largest of slot s's ncopies (<= 64) copies, as the double its
// bit pattern is, then out[nslots] = *extra (0 without one).  One wavefront
// per slot (workgroup s); out is pinned host memory the host reads after
// synchronising.
__global__ void __launch_bounds__(64) k_pack_slots(const unsigned long long *__restrict__ slots,
                                                   int nslots, int ncopies,
                                                   const double *__restrict__ extra, double *out) {
  const int s = blockIdx.x, c = threadIdx.x;
  unsigned long long m = c < ncopies ? slots[(size_t)s * ncopies + c] : 0ull;
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if (c == 0) {
    out[s] = __longlong_as_double((long long)m);
    if (s == 0) out[nslots] = extra ? *extra : 0.0;
  }
}

__global__ void __launch_bounds__(256) k_maxabs(const double *x, int64_t n, unsigned long long *slot) {
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v = fmax(v, fabs(x[i]));
  wave_slot_max(slot, 0, v);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <typename Tin, typename Tout>
hipError_t launch_pass(hipStream_t st, const Tin *in, Dims in_dims, int ax, const Ell &op,
                       Tout *out, int epi, const double *sub, unsigned long long *slots,
                       int slot_base, const int *gid, int gaxis) {
  Dims od = in_dims;
  od.d[ax] = op.R;
  if (od.total() == 0) return hipSuccess;
  if (od.d[0] > 65535 || od.d[1] > 65535 || od.total() >= (1LL << 31) ||
      in_dims.total() >= (1LL << 31))
    return hipErrorInvalidValue;
  const int bs = od.d[2] >= 256 ? 256 : (int)((od.d[2] + 63) / 64) * 64;
  const dim3 grid(nblk(od.d[2], bs), (unsigned)od.d[1], (unsigned)od.d[0]);
  const int o0 = (int)od.d[0], o1 = (int)od.d[1], o2 = (int)od.d[2], rin = (int)in_dims.d[ax];
  switch (epi) {
    case EPI_STORE:
      k_pass<Tin, Tout, EPI_STORE><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op, slots,
                                                         slot_base, gid, gaxis);
      break;
    case EPI_SUBFROM:
      k_pass<Tin, Tout, EPI_SUBFROM><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op,
                                                           slots, slot_base, gid, gaxis);
      break;
    case EPI_STOREMAX:
      k_pass<Tin, Tout, EPI_STOREMAX><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op,
                                                           slots, slot_base, gid, gaxis);
      break;
    case EPI_ADDTO:
      k_pass<Tin, Tout, EPI_ADDTO><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op, slots,
                                                         slot_base, gid, gaxis);
      break;
    case EPI_RESID32:
      k_pass<Tin, Tout, EPI_RESID32><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op,
                                                           slots, slot_base, gid, gaxis);
      break;
    case EPI_RESID64:
      k_pass<Tin, Tout, EPI_RESID64><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op,
                                                           slots, slot_base, gid, gaxis);
      break;
    default:
      k_pass<Tin, Tout, EPI_MAXABS><<<grid, bs, 0, st>>>(in, out, sub, o0, o1, o2, ax, rin, op, slots,
                                                          slot_base, gid, gaxis);
      break;
  }
  return hipGetLastError();
}

template hipError_t launch_pass<double, double>(hipStream_t, const double *, Dims, int, const Ell &,
                                                double *, int, const double *, unsigned long long *,
                                                int, const int *, int);
template hipError_t launch_pass<float, double>(hipStream_t, const float *, Dims, int, const Ell &,
                                               double *, int, const double *, unsigned long long *,
                                               int, const int *, int);
template hipError_t launch_pass<double, float>(hipStream_t, const double *, Dims, int, const Ell &,
                                               float *, int, const double *, unsigned long long *,
                                               int, const int *, int);
template hipError_t launch_pass<float, float>(hipStream_t, const float *, Dims, int, const Ell &,
                                              float *, int, const double *, unsigned long long *,
                                              int, const int *, int);

template <typename TQ>
hipError_t launch_box_resid(hipStream_t st, const TQ *q, Dims qd, double *r, Dims rd,
                            const int *qm0, const int *qm1, const int *qm2) {
  if (rd.total() == 0) return hipSuccess;
  const int bs = rd.d[2] >= 256 ? 256 : (int)((rd.d[2] + 63) / 64) * 64;
  const dim3 grid(nblk(rd.d[2], bs), (unsigned)rd.d[1], (unsigned)rd.d[0]);
  k_box_resid<TQ><<<grid, bs, 0, st>>>(q, (int)qd.d[1], (int)qd.d[2], r, (int)rd.d[0], (int)rd.d[1],
                                       (int)rd.d[2], qm0, qm1, qm2);
  return hipGetLastError();
}
template hipError_t launch_box_resid<float>(hipStream_t, const float *, Dims, double *, Dims,
                                            const int *, const int *, const int *);
template hipError_t launch_box_resid<double>(hipStream_t, const double *, Dims, double *, Dims,
                                             const int *, const int *, const int *);

hipError_t launch_fill(hipStream_t st, double *x, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  k_fill<<<nblk(n, 256), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_slots(hipStream_t st, unsigned long long *slots, int n, double *hist, int idx,
                             const unsigned long long *from) {
  static_assert(kSlotMaxDP == 0 && kSlotCopies == 64, "one wavefront reads the max-correction slot");
  k_zero_slots<<<nblk(n, 64), 64, 0, st>>>(slots, n, hist, idx, from ? from : slots);
  return hipGetLastError();
}

hipError_t launch_pack_slots(hipStream_t st, const unsigned long long *slots, int nslots, int ncopies,
                             const double *extra, double *out) {
  if (nslots < 1 || ncopies < 1 || ncopies > 64) return hipErrorInvalidValue;
  k_pack_slots<<<nslots, 64, 0, st>>>(slots, nslots, ncopies, extra, out);
  return hipGetLastError();
}

hipError_t launch_maxabs(hipStream_t st, const double *x, int64_t n, unsigned long long *slot) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(nblk(n, 256), 2048);
  k_maxabs<<<grid, 256, 0, st>>>(x, n, slot);
  return hipGetLastError();
}

}  // namespace mfa
