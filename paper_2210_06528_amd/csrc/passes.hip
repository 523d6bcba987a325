// Generic axis pass: apply a row-sparse operator along one axis of a 3-D
// array (the building block of every tensor-product contraction here), with
// an epilogue that stores, forms a residual, accumulates into the control
// points or only reduces max |value| into a slot.
#include "mfa_internal.hpp"

namespace mfa {

namespace {

__device__ __forceinline__ void slot_max(unsigned long long *slots, int slot, double v) {
  atomicMax(slots + slot, (unsigned long long)__double_as_longlong(v));
}

// Wavefront max of v (non-negative) into `slot`; lanes with different slots
// fall back to one atomic each.
__device__ __forceinline__ void wave_slot_max(unsigned long long *slots, int slot, double v) {
  const int s0 = __shfl(slot, 0, 64);
  if (__all(slot == s0)) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) slot_max(slots, s0, v);
  } else {
    slot_max(slots, slot, v);
  }
}

template <typename Tin, typename Tout, int EPI>
__global__ void __launch_bounds__(256) k_pass(const Tin *__restrict__ in, Tout *__restrict__ out,
                                              const double *__restrict__ sub, int64_t o0,
                                              int64_t o1, int64_t o2, int ax, int64_t rin, Ell op,
                                              unsigned long long *slots, int slot_base,
                                              const int *__restrict__ gid, int gaxis) {
  const int64_t total = o0 * o1 * o2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = idx < total;
  double acc = 0.0;
  int slot = slot_base;
  if (valid) {
    int64_t x[3];
    x[2] = idx % o2;
    const int64_t t = idx / o2;
    x[1] = t % o1;
    x[0] = t / o1;
    const int64_t row = x[ax];
    if (EPI == EPI_MAXABS && gid != nullptr) slot = slot_base + gid[x[gaxis]];
    const int64_t i1 = ax == 1 ? rin : o1;
    const int64_t i2 = ax == 2 ? rin : o2;
    const int64_t stride = ax == 2 ? 1 : (ax == 1 ? i2 : i1 * i2);
    x[ax] = 0;
    const int64_t base = (x[0] * i1 + x[1]) * i2 + x[2];
    const int *cl = op.col + row * op.L;
    const double *vl = op.val + row * op.L;
    const int ln = op.len[row];
    for (int q = 0; q < ln; ++q) acc += vl[q] * (double)in[base + (int64_t)cl[q] * stride];
    if (EPI == EPI_STORE) {
      out[idx] = (Tout)acc;
    } else if (EPI == EPI_SUBFROM) {
      acc = sub[idx] - acc;
      out[idx] = (Tout)acc;
    } else if (EPI == EPI_ADDTO) {
      out[idx] = (Tout)((double)out[idx] + acc);
    }
  }
  if (EPI != EPI_STORE) wave_slot_max(slots, slot, valid ? fabs(acc) : 0.0);
}

__global__ void k_fill(double *x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_zero_slots(unsigned long long *s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = 0ull;
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
  const int64_t total = od.total();
  if (total == 0) return hipSuccess;
  const unsigned grid = nblk(total, 256);
  const int64_t rin = in_dims.d[ax];
  switch (epi) {
    case EPI_STORE:
      k_pass<Tin, Tout, EPI_STORE><<<grid, 256, 0, st>>>(in, out, sub, od.d[0], od.d[1], od.d[2], ax,
                                                         rin, op, slots, slot_base, gid, gaxis);
      break;
    case EPI_SUBFROM:
      k_pass<Tin, Tout, EPI_SUBFROM><<<grid, 256, 0, st>>>(in, out, sub, od.d[0], od.d[1], od.d[2],
                                                           ax, rin, op, slots, slot_base, gid, gaxis);
      break;
    case EPI_ADDTO:
      k_pass<Tin, Tout, EPI_ADDTO><<<grid, 256, 0, st>>>(in, out, sub, od.d[0], od.d[1], od.d[2], ax,
                                                         rin, op, slots, slot_base, gid, gaxis);
      break;
    default:
      k_pass<Tin, Tout, EPI_MAXABS><<<grid, 256, 0, st>>>(in, out, sub, od.d[0], od.d[1], od.d[2], ax,
                                                          rin, op, slots, slot_base, gid, gaxis);
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

hipError_t launch_fill(hipStream_t st, double *x, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  k_fill<<<nblk(n, 256), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_slots(hipStream_t st, unsigned long long *slots, int n) {
  k_zero_slots<<<nblk(n, 64), 64, 0, st>>>(slots, n);
  return hipGetLastError();
}

hipError_t launch_maxabs(hipStream_t st, const double *x, int64_t n, unsigned long long *slot) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(nblk(n, 256), 2048);
  k_maxabs<<<grid, 256, 0, st>>>(x, n, slot);
  return hipGetLastError();
}

}  // namespace mfa
