// C ABI of the MFA encoder: handle lifecycle, Schwarz sweeps, encode loop,
// decode and inspection.  See include/mfa.h for the contract of each call.
#include <algorithm>
#include <tuple>
#include <mutex>
#include <map>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include <hip/hip_bf16.h>

#include <cstdlib>

#include "mfa_internal.hpp"

using namespace mfa;

struct mfa_handle {
  Handle h;
};

namespace mfa {

Handle::~Handle() {
  for (auto &v : ev_used)
    for (auto &pr : v) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (auto e : ev_pool) hipEventDestroy(e);
}

static hipEvent_t take_event(Handle &h) {
  if (!h.ev_pool.empty()) {
    hipEvent_t e = h.ev_pool.back();
    h.ev_pool.pop_back();
    return e;
  }
  // Timing events only take timestamps: nothing reads device memory through
  // them (the host reads results after a stream synchronisation), so they
  // skip the system-scope release a default event record performs, an L2
  // writeback and invalidate that left the GPU idle for about 5 us on each
  // side of a timed launch and made the launch after it start from cold caches.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

TimeScope::TimeScope(Handle &hh, int c) : h(hh), cls(c) {
  if (!(h.timing & (1 << c))) return;
  if (h.timing_seen[c]++ % h.timing_every != h.timing_first) return;
  e0 = take_event(h);
  e1 = take_event(h);
  if (e0) hipEventRecord(e0, h.stream);
}

TimeScope::~TimeScope() {
  if (!e0 || !e1) return;
  hipEventRecord(e1, h.stream);
  h.ev_used[cls].push_back({e0, e1});
}

}  // namespace mfa

namespace {

thread_local std::string g_last_error;

mfa_status fail(mfa_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

mfa_status hip_fail(hipError_t e, const char *where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return MFA_EDEVICE;
}

#define HIP_CHECK(x, where)                  \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

Dims ctrl_dims(const Handle &h) { return Dims{{h.ax[0].n, h.ax[1].n, h.ax[2].n}}; }
// control grid of the model the handle encodes (the variants' own layouts)
Dims model_dims(const Handle &h) {
  if (!h.variant) return ctrl_dims(h);
  return Dims{{h.ax[0].nv, h.ax[1].nv, h.ax[2].nv}};
}
Dims data_dims(const Handle &h) { return Dims{{h.ax[0].m, h.ax[1].m, h.ax[2].m}}; }

struct Step {
  int ax;
  const Ell *op;
};

// Apply `steps` in order starting from `in` (dims `d`); intermediates
// alternate between the two scratch buffers; the last step uses `epi` and
// writes `out` (or only reduces).
template <typename Tin, typename Tout>
hipError_t run_chain(Handle &h, const Tin *in, Dims d, const std::vector<Step> &steps, Tout *out,
                     int epi, const double *sub, int slot_base, const int *gid, int gaxis,
                     double *bufA, double *bufB) {
  if (steps.empty()) return hipSuccess;
  if (steps.size() == 1)
    return launch_pass<Tin, Tout>(h.stream, in, d, steps[0].ax, *steps[0].op, out, epi, sub, h.slots,
                                  slot_base, gid, gaxis);
  double *bufs[2] = {bufA, bufB};
  {
    // every intermediate must fit the scratch buffer it goes to
    const int64_t cap[2] = {bufA == h.s1 ? h.s1n : h.s2n, bufB == h.s2 ? h.s2n : h.s1n};
    Dims t = d;
    for (size_t s = 0; s + 1 < steps.size(); ++s) {
      t.d[steps[s].ax] = steps[s].op->R;
      if (t.total() > cap[s & 1]) return hipErrorInvalidValue;
    }
  }
  int w = 0;
  hipError_t e = launch_pass<Tin, double>(h.stream, in, d, steps[0].ax, *steps[0].op, bufs[w],
                                          EPI_STORE, nullptr, h.slots, 0, nullptr, 0);
  if (e != hipSuccess) return e;
  d.d[steps[0].ax] = steps[0].op->R;
  for (size_t s = 1; s + 1 < steps.size(); ++s) {
    e = launch_pass<double, double>(h.stream, bufs[w], d, steps[s].ax, *steps[s].op, bufs[w ^ 1],
                                    EPI_STORE, nullptr, h.slots, 0, nullptr, 0);
    if (e != hipSuccess) return e;
    d.d[steps[s].ax] = steps[s].op->R;
    w ^= 1;
  }
  return launch_pass<double, Tout>(h.stream, bufs[w], d, steps.back().ax, *steps.back().op, out, epi,
                                   sub, h.slots, slot_base, gid, gaxis);
}

// c = N^T Q (every active axis, innermost first)
template <typename T>
hipError_t project(Handle &h, const T *q) {
  TimeScope ts(h, MFA_K_PROJECT);
  if (grid_pass_ok(h)) {
    hipError_t e = launch_project_grid(h, q, sizeof(T) == sizeof(float));
    if (e != hipErrorNotSupported) return e;
  }
  std::vector<Step> st;
  for (int a = 2; a >= 0; --a)
    if (h.ax[a].active) st.push_back({a, &h.ax[a].NT});
  return run_chain<T, double>(h, q, data_dims(h), st, h.c, EPI_STORE, nullptr, 0, nullptr, 0, h.s1,
                              h.s2);
}

bool mfma_ok(const Handle &h) {
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active && !mfma_fits(h.ax[a].npad)) return false;
  return true;
}

bool fast_sweep_ok(const Handle &h, size_t elem) {
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active && !bsolve_seg_ok(h.ax[a]) && bsolve_lds(h.ax[a].Fmax, h.p, elem) > 64 * 1024)
      return false;
  return true;
}

// Schwarz correction along every active axis with the banded-solve kernel;
// the last axis adds the combined correction into P.
template <typename T>
hipError_t correct_bsolve(Handle &h, const T *g) {
  const int n0 = h.ax[0].n, n1 = h.ax[1].n, n2 = h.ax[2].n;
  // contiguous axis first: the last pass (which adds into P) then runs on a
  // strided axis where the lanes of a wavefront touch consecutive addresses
  int act[3], na = 0;
  for (int a = 2; a >= 0; --a)
    if (h.ax[a].active) act[na++] = a;
  const T *in = g;
  T *bufs[2] = {reinterpret_cast<T *>(h.s1), reinterpret_cast<T *>(h.s2)};
  for (int i = 0; i < na; ++i) {
    const Axis &X = h.ax[act[i]];
    const bool last = i == na - 1;
    T *out = last ? nullptr : bufs[i & 1];
    TimeScope ts(h, MFA_K_CORRECT);
    hipError_t e = launch_bsolve<T, T, T>(h.stream, in, out, last ? h.P : nullptr, act[i], n0, n1, n2,
                                          h.p, X, h.combine, h.slots);
    if (e != hipSuccess) return e;
    in = out;
  }
  return hipSuccess;
}

// Autotuned choice between the fused axis-2/axis-1 split-BF16 correction and
// the two separate passes.  Both map g to the same intermediate s1 with the
// same arithmetic (bitwise equal) and neither touches P or the reduction
// slots, so for a large shape the first sweep times both on the live arrays
// (three runs each, HIP events, fastest kept) and the choice is cached per
// shape class for the process: the padded band widths of axes 1 and 2, the
// degree, the combine rule and axis 0's length in steps of 32.  A candidate
// replaces the fused default only if it is at least 10% faster.  Small
// shapes, handles without auxiliary objects (no-allocation) and event-timed
// runs take the fused default untimed.
struct CorrKey {
  int np1, np2, p, comb, n0c;
  bool operator<(const CorrKey &o) const {
    return std::tie(np1, np2, p, comb, n0c) < std::tie(o.np1, o.np2, o.p, o.comb, o.n0c);
  }
};
std::mutex g_corr_mu;
std::map<CorrKey, bool> g_corr_fused;
constexpr int64_t kCorrTuneMin = 1 << 20;

hipError_t separate21(Handle &h, const float *gf, float *s1, float *s2) {
  hipError_t e = launch_mfma_correct(h, 2, gf, s2, false);
  if (e != hipSuccess) return e;
  return launch_mfma_correct(h, 1, s2, s1, false);
}

hipError_t choose_fused21(Handle &h, const float *gf, bool *fused) {
  *fused = h.fuse21 && h.ax[0].active && mfma_fused21_ok(h);
  if (!*fused || h.nctrl_total < kCorrTuneMin || h.serial || h.timing) return hipSuccess;
  const CorrKey key{h.ax[1].npad, h.ax[2].npad, h.p, h.combine, (h.ax[0].n + 31) / 32};
  {
    std::lock_guard<std::mutex> lk(g_corr_mu);
    auto it = g_corr_fused.find(key);
    if (it != g_corr_fused.end()) {
      *fused = it->second;
      return hipSuccess;
    }
  }
  float *s1 = reinterpret_cast<float *>(h.s1), *s2 = reinterpret_cast<float *>(h.s2);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return hipErrorOutOfMemory;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return hipErrorOutOfMemory;
  }
  float best[2] = {1e30f, 1e30f};
  hipError_t err = hipSuccess;
  for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
    for (int c = 0; c < 2 && err == hipSuccess; ++c) {
      hipEventRecord(e0, h.stream);
      err = c == 0 ? launch_mfma_fused21(h, gf, s1) : separate21(h, gf, s1, s2);
      hipEventRecord(e1, h.stream);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && rep > 0) best[c] = std::min(best[c], ms);   // rep 0 warms up
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return err;
  *fused = !(best[1] < 0.9f * best[0]);
  std::lock_guard<std::mutex> lk(g_corr_mu);
  g_corr_fused[key] = *fused;
  return hipSuccess;
}

// One sweep (NORMAL right-hand side):
//   g = c - (A_0 x A_1 x A_2) P      (the local residuals N_F^T (Q - N P) of all
//                                     subdomains at once)
//   P += (M_0 x M_1 x M_2) g         (local solves with lagged ghosts and the
//                                     1/n_s combine, Section 2.3.2)
// The residual g = c - A P of a sweep: the stencil kernel, or, when P = 0
// (p_zero: the first sweep of a cold start), g = c (the stencil of zeros is
// zero), which needs no stencil and no bookkeeping turn (both slot sets are
// clear and no correction history exists yet).  Only the stencil kernel's
// launches are timed as the residual class.
template <typename TG>
static hipError_t residual(Handle &h, TG *g, const SlotTurn &turn, bool p_zero) {
  if (p_zero) return launch_resid_zero<TG>(h.stream, h.c, g, h.nctrl_total, h.slots);
  TimeScope ts(h, MFA_K_RESID);
  return launch_resid<TG>(h.stream, h.p, h.P, h.c, g, h.ax[0].d_acoef, h.ax[1].d_acoef, h.ax[2].d_acoef,
                          h.ax[0].n, h.ax[1].n, h.ax[2].n, h.slots, turn, !h.serial);
}

hipError_t sweep_normal(Handle &h, const SlotTurn &turn, bool p_zero) {
  if (h.precision == MFA_PREC_MIXED_BF16 && mfma_ok(h)) {
    // residual in float64, rounded to FP32; correction on the matrix cores
    h.g_type = 1;
    float *gf = reinterpret_cast<float *>(h.g);
    hipError_t e = residual<float>(h, gf, turn, p_zero);
    if (e != hipSuccess) return e;
    bool fused = false;
    if ((e = choose_fused21(h, gf, &fused)) != hipSuccess) return e;
    if (fused) {
      // axes 2 and 1 in one pass, then axis 0 adds into P
      float *s1 = reinterpret_cast<float *>(h.s1);
      {
        TimeScope ts(h, MFA_K_CORRECT);
        e = launch_mfma_fused21(h, gf, s1);
      }
      if (e != hipSuccess) return e;
      TimeScope ts(h, MFA_K_CORRECT);
      return launch_mfma_correct(h, 0, s1, nullptr, true);
    }
    int act[3], na = 0;
    for (int a = 2; a >= 0; --a)
      if (h.ax[a].active) act[na++] = a;
    const float *in = gf;
    float *bufs[2] = {reinterpret_cast<float *>(h.s1), reinterpret_cast<float *>(h.s2)};
    for (int i = 0; i < na; ++i) {
      const bool last = i == na - 1;
      float *out = last ? nullptr : bufs[i & 1];
      TimeScope ts(h, MFA_K_CORRECT);
      e = launch_mfma_correct(h, act[i], in, out, last);
      if (e != hipSuccess) return e;
      in = out;
    }
    return hipSuccess;
  }
  const bool low = h.precision != MFA_PREC_FP64;
  if (fast_sweep_ok(h, low ? sizeof(float) : sizeof(double))) {
    h.g_type = low ? 1 : 0;
    if (low) {
      float *gf = reinterpret_cast<float *>(h.g);
      hipError_t e = residual<float>(h, gf, turn, p_zero);
      if (e != hipSuccess) return e;
      return correct_bsolve<float>(h, gf);
    }
    hipError_t e = residual<double>(h, h.g, turn, p_zero);
    if (e != hipSuccess) return e;
    return correct_bsolve<double>(h, h.g);
  }
  // general path: row-sparse operator passes (any segment length)
  h.g_type = 0;
  std::vector<Step> st;
  for (int a = 2; a >= 0; --a)
    if (h.ax[a].active) st.push_back({a, &h.ax[a].A});
  hipError_t e = run_chain<double, double>(h, h.P, ctrl_dims(h), st, h.g, EPI_SUBFROM, h.c,
                                           kSlotNres, nullptr, 0, h.s1, h.s2);
  if (e != hipSuccess) return e;
  st.clear();
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active) st.push_back({a, &h.ax[a].M});
  return run_chain<double, double>(h, h.g, ctrl_dims(h), st, h.P, EPI_ADDTO, nullptr, kSlotMaxDP,
                                   nullptr, 0, h.s1, h.s2);
}

// One sweep with the DATABOX right-hand side, as Algorithm 1 is written:
// decode the current spline on every subdomain's data box (segmented layout,
// one segment per subdomain and axis), residual against Q, contract with the
// local N_F^T, apply the local inverses, combine into P.  On check sweeps the
// interface jumps are evaluated from the local right-hand sides.
hipError_t sweep_databox(Handle &h, bool metrics) {
  Dims d = ctrl_dims(h);
  double *buf[2] = {h.b1, h.b2};
  int w = 0;
  const double *cur = h.P;
  hipError_t e;
  auto pass = [&](int a, const Ell &op, int epi, double *out, int slot) {
    e = launch_pass<double, double>(h.stream, cur, d, a, op, out, epi, nullptr, h.slots, slot,
                                    nullptr, 0);
    d.d[a] = op.R;
    cur = out;
  };
  for (int a = 2; a >= 0; --a) {
    if (!h.ax[a].active) continue;
    pass(a, h.ax[a].Nseg, EPI_STORE, buf[w], 0);
    if (e != hipSuccess) return e;
    w ^= 1;
  }
  // point residual on the boxes
  double *rbox = const_cast<double *>(cur);
  e = h.q_dtype == MFA_F32
          ? launch_box_resid<float>(h.stream, reinterpret_cast<const float *>(h.q), data_dims(h), rbox,
                                    d, h.ax[0].d_qmap, h.ax[1].d_qmap, h.ax[2].d_qmap)
          : launch_box_resid<double>(h.stream, reinterpret_cast<const double *>(h.q), data_dims(h),
                                     rbox, d, h.ax[0].d_qmap, h.ax[1].d_qmap, h.ax[2].d_qmap);
  if (e != hipSuccess) return e;
  int last = -1;
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active) last = a;
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active) continue;
    pass(a, h.ax[a].NsegT, a == last ? EPI_STOREMAX : EPI_STORE, buf[w], kSlotNres);
    if (e != hipSuccess) return e;
    w ^= 1;
  }
  if (metrics) {
    // jumps from the local right-hand sides (segmented layout)
    const Dims rd = d;
    for (int a = 0; a < 3; ++a) {
      if (!h.ax[a].active || h.ax[a].B < 2) continue;
      std::vector<Step> st{{a, &h.ax[a].Jseg}};
      for (int c = 0; c < 3; ++c)
        if (c != a && h.ax[c].active) st.push_back({c, &h.ax[c].Omseg});
      e = run_chain<double, double>(h, cur, rd, st, (double *)nullptr, EPI_MAXABS, nullptr,
                                    kSlotJ + a * kMaxP, h.ax[a].d_gidJ, a, h.s1, h.s2);
      if (e != hipSuccess) return e;
    }
  }
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active) continue;
    pass(a, h.ax[a].Zseg, EPI_STORE, buf[w], 0);
    if (e != hipSuccess) return e;
    w ^= 1;
  }
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active) continue;
    if (a == last) {
      pass(a, h.ax[a].Comb, EPI_ADDTO, h.P, kSlotMaxDP);
    } else {
      pass(a, h.ax[a].Comb, EPI_STORE, buf[w], 0);
      w ^= 1;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Two auxiliary streams (default priority) and fork/join events per host
// thread and device, created on first use and kept for the life of the
// process: concurrent handles on different threads never share them.
struct AuxStreams {
  hipStream_t s[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};

double *pinned_block(int device) {
  static thread_local double *per_dev[16] = {};
  static thread_local bool tried[16] = {};
  if (device < 0 || device >= 16) return nullptr;
  if (!tried[device]) {
    tried[device] = true;
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(double) * kPinnedDoubles, hipHostMallocDefault) == hipSuccess)
      per_dev[device] = static_cast<double *>(p);
  }
  return per_dev[device];
}

static AuxStreams *aux_streams(int device) {
  static thread_local AuxStreams per_dev[16];
  if (device < 0 || device >= 16) return nullptr;
  AuxStreams &a = per_dev[device];
  if (!a.fork) {
    for (int i = 0; i < 2; ++i) {
      if (hipStreamCreateWithFlags(&a.s[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
      if (hipEventCreateWithFlags(&a.join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
    }
    if (hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
  }
  return &a;
}

// Runs a launch helper on another stream: the helpers launch on h.stream.
struct StreamSwap {
  Handle &h;
  hipStream_t saved;
  StreamSwap(Handle &hh, hipStream_t s) : h(hh), saved(hh.stream) { h.stream = s; }
  ~StreamSwap() { h.stream = saved; }
};

// Jump of the interfaces along axis a: the interface functionals applied to
// the residual into U, then expanded over the other axes.
static hipError_t jump_axis(Handle &h, int a, double *U) {
  hipError_t e =
      h.g_type == 1   ? launch_jump_project<float>(h, a, reinterpret_cast<const float *>(h.g), U)
      : h.g_type == 2 ? launch_jump_project<__hip_bfloat16>(
                            h, a, reinterpret_cast<const __hip_bfloat16 *>(h.g), U)
                      : launch_jump_project<double>(h, a, h.g, U);
  if (e != hipSuccess) return e;
  return launch_jump_expand(h, a, U);
}

// Jump and scale reductions of the sweep just done (g still holds the
// residual the sweep used; P holds the new consensus).  The per-axis jump
// chains and the derivative scales are independent latency-bound kernels
// whose maxima go to separate slots: axis 0 and the scales run on the
// caller's stream, axes 1 and 2 on the two auxiliary streams (forked from it
// and joined back), each axis with its own part of the scratch array s1.
hipError_t sweep_metrics(Handle &h) {
  TimeScope ts(h, MFA_K_METRICS);
  int64_t off[3] = {0, 0, 0}, tot = 0;
  bool jumps[3] = {false, false, false};
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active || h.ax[a].B < 2) continue;
    jumps[a] = true;
    off[a] = tot;
    tot += (int64_t)(h.ax[a].B - 1) * h.p * (h.nctrl_total / h.ax[a].n);
  }
  AuxStreams *aux = (tot <= h.s1n && !h.serial) ? aux_streams(h.device) : nullptr;
  if (!aux) {
    for (int a = 0; a < 3; ++a) {
      if (!jumps[a]) continue;
      hipError_t e = jump_axis(h, a, h.s1);
      if (e != hipSuccess) return e;
    }
    return launch_deriv_scale(h);
  }
  hipError_t e = hipEventRecord(aux->fork, h.stream);
  if (e != hipSuccess) return e;
  for (int a = 1; a < 3; ++a) {
    if (!jumps[a]) continue;
    hipStream_t st = aux->s[a - 1];
    if ((e = hipStreamWaitEvent(st, aux->fork, 0)) != hipSuccess) return e;
    {
      StreamSwap sw(h, st);
      if ((e = jump_axis(h, a, h.s1 + off[a])) != hipSuccess) return e;
    }
    if ((e = hipEventRecord(aux->join[a - 1], st)) != hipSuccess) return e;
  }
  if (jumps[0] && (e = jump_axis(h, 0, h.s1 + off[0])) != hipSuccess) return e;
  if ((e = launch_deriv_scale(h)) != hipSuccess) return e;
  for (int a = 1; a < 3; ++a)
    if (jumps[a] && (e = hipStreamWaitEvent(h.stream, aux->join[a - 1], 0)) != hipSuccess) return e;
  return hipSuccess;
}

// Algorithm 1's error E = Q - N P at the current control points: one decode
// of the spline on the data grid compared with the data of the last encode
// or step, reduced to max |E| and ||E||_2 (nothing is stored).
mfa_status residual_stats(Handle &h, double *res_max, double *res_l2) {
  const int nres = 2 * kSlotCopies;
  hipError_t e = launch_zero_slots(h.stream, h.res_slots, nres);
  if (e != hipSuccess) return hip_fail(e, "residual");
  const bool f32 = h.q_dtype == MFA_F32;
  bool done = false;
  if (grid_pass_ok(h) && !h.variant) {
    const int r[3] = {0, 0, 0};
    e = launch_decode_grid(h, const_cast<void *>(h.q), f32, r, h.res_slots);
    if (e == hipSuccess) done = true;
    else if (e != hipErrorNotSupported) return hip_fail(e, "residual");
  }
  if (!done) {
    std::vector<Step> st;
    for (int a = 2; a >= 0; --a)
      if (h.ax[a].active) st.push_back({a, h.variant ? &h.ax[a].Nv[0] : &h.ax[a].N[0]});
    unsigned long long *saved = h.slots;
    h.slots = h.res_slots;   // the last pass reduces into the residual slots
    e = run_chain<double, double>(h, h.P, model_dims(h), st, (double *)nullptr,
                                  f32 ? EPI_RESID32 : EPI_RESID64, (const double *)h.q, 0, nullptr,
                                  0, h.s1, h.s2);
    h.slots = saved;
    if (e != hipSuccess) return hip_fail(e, "residual");
  }
  std::vector<unsigned long long> raw(nres);
  HIP_CHECK(hipMemcpyAsync(raw.data(), h.res_slots, sizeof(unsigned long long) * nres,
                           hipMemcpyDeviceToHost, h.stream), "residual");
  HIP_CHECK(hipStreamSynchronize(h.stream), "residual");
  unsigned long long mx = 0;
  double sq = 0.0;
  for (int c = 0; c < kSlotCopies; ++c) {
    mx = std::max(mx, raw[c]);
    double v;
    std::memcpy(&v, &raw[kSlotCopies + c], sizeof(v));
    sq += v;
  }
  std::memcpy(res_max, &mx, sizeof(double));
  *res_l2 = std::sqrt(sq);
  return MFA_OK;
}

// One-shot fit of the DECOUPLED / CLAMPED variants: P = (L_0 x L_1 x L_2) Q
// through the pass chain, then max |P| and the interface jumps of the model
// (rows along the interface axis, decode rows on the others), normalised by
// max |P|.
mfa_status encode_variant(Handle &h, mfa_step_stats *out) {
  const int64_t nset = (int64_t)kNumSlots * kSlotCopies;
  h.slots = h.slot_base;
  hipError_t e = launch_zero_slots(h.stream, h.slots, (int)nset);
  if (e != hipSuccess) return hip_fail(e, "zero slots");
  std::vector<Step> st;
  for (int a = 2; a >= 0; --a)
    if (h.ax[a].active) st.push_back({a, &h.ax[a].Lv});
  e = h.q_dtype == MFA_F32
          ? run_chain<float, double>(h, (const float *)h.q, data_dims(h), st, h.P, EPI_STORE, nullptr,
                                     0, nullptr, 0, h.s1, h.s2)
          : run_chain<double, double>(h, (const double *)h.q, data_dims(h), st, h.P, EPI_STORE,
                                      nullptr, 0, nullptr, 0, h.s1, h.s2);
  if (e != hipSuccess) return hip_fail(e, "variant fit");
  if ((e = launch_maxabs(h.stream, h.P, h.nctrl_total, h.slots + (size_t)kSlotCtrl * kSlotCopies)) !=
      hipSuccess)
    return hip_fail(e, "variant fit");
  const Dims md = model_dims(h);
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active || h.ax[a].B < 2) continue;
    std::vector<Step> js{{a, &h.ax[a].Jv}};
    for (int c = 0; c < 3; ++c)
      if (c != a && h.ax[c].active) js.push_back({c, &h.ax[c].Nv[0]});
    e = run_chain<double, double>(h, h.P, md, js, (double *)nullptr, EPI_MAXABS, nullptr,
                                  kSlotJ + a * kMaxP, h.ax[a].d_gidJ, a, h.s1, h.s2);
    if (e != hipSuccess) return hip_fail(e, "variant jumps");
  }
  std::vector<unsigned long long> raw((size_t)kNumSlots * kSlotCopies);
  HIP_CHECK(hipMemcpyAsync(raw.data(), h.slots, sizeof(unsigned long long) * raw.size(),
                           hipMemcpyDeviceToHost, h.stream), "variant stats");
  HIP_CHECK(hipStreamSynchronize(h.stream), "variant stats");
  auto val = [&](int s) {
    unsigned long long m = 0;
    for (int c = 0; c < kSlotCopies; ++c) m = std::max(m, raw[(size_t)s * kSlotCopies + c]);
    double d;
    std::memcpy(&d, &m, sizeof(d));
    return d;
  };
  mfa_step_stats s{};
  s.sweep = 1;
  s.converged = 1;
  s.ctrl_max = val(kSlotCtrl);
  s.max_dP = s.ctrl_max;
  s.nres_max = 0.0;
  s.res_max = s.res_l2 = std::numeric_limits<double>::quiet_NaN();
  bool fin = std::isfinite(s.ctrl_max);
  for (int r = 0; r < h.p; ++r) {
    double jr = 0.0;
    for (int a = 0; a < 3; ++a) {
      if (!h.ax[a].active || h.ax[a].B < 2) continue;
      const double rj = val(kSlotJ + a * kMaxP + r);
      if (!std::isfinite(rj)) fin = false;
      jr = std::max(jr, s.ctrl_max > 0.0 ? rj / s.ctrl_max : 0.0);
    }
    s.jump[r] = jr;
  }
  h.sweep = 1;
  if (out) *out = s;
  if (!fin) return fail(MFA_ENOTCONV, "non-finite value in the fit");
  return MFA_OK;
}

// hist_val (optional): h.hist[hist_idx] copied back with the slots, under the
// same synchronisation.
mfa_status read_stats(Handle &h, mfa_step_stats *out, double jump_tol, bool *finite,
                      double *hist_val = nullptr, int hist_idx = 0) {
  static_assert(kNumSlots + 1 <= kPinnedDoubles, "the slot maxima fit the pinned block");
  // non-negative doubles order like their bit patterns (NaN sorts above inf):
  // a slot's value is the largest bit pattern of its copies
  std::vector<double> vals(kNumSlots);
  // handles without allocations copy to pageable memory; the others have the
  // slots reduced on the device into this thread's pinned block
  double *pin = h.noalloc_gen ? nullptr : pinned_block(h.device);
  if (pin) {
    HIP_CHECK(launch_pack_slots(h.stream, h.slots, kNumSlots, kSlotCopies,
                                hist_val ? h.hist + hist_idx : nullptr, pin),
              "read stats");
    HIP_CHECK(hipStreamSynchronize(h.stream), "read stats");
    for (int s = 0; s < kNumSlots; ++s) vals[s] = pin[s];
    if (hist_val) *hist_val = pin[kNumSlots];
  } else {
    std::vector<unsigned long long> raw((size_t)kNumSlots * kSlotCopies);
    HIP_CHECK(hipMemcpyAsync(raw.data(), h.slots, sizeof(unsigned long long) * raw.size(),
                             hipMemcpyDeviceToHost, h.stream), "read stats");
    if (hist_val)
      HIP_CHECK(hipMemcpyAsync(hist_val, h.hist + hist_idx, sizeof(double), hipMemcpyDeviceToHost, h.stream),
                "read correction history");
    HIP_CHECK(hipStreamSynchronize(h.stream), "read stats");
    for (int s = 0; s < kNumSlots; ++s) {
      unsigned long long m = 0;
      for (int c = 0; c < kSlotCopies; ++c) m = std::max(m, raw[(size_t)s * kSlotCopies + c]);
      std::memcpy(&vals[s], &m, sizeof(double));
    }
  }
  auto val = [&](int s) { return vals[s]; };
  mfa_step_stats st{};
  st.sweep = h.sweep;
  st.res_max = st.res_l2 = std::numeric_limits<double>::quiet_NaN();
  st.max_dP = val(kSlotMaxDP);
  st.nres_max = val(kSlotNres);
  double s0 = 0.0;
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active) s0 = std::max(s0, val(kSlotS + a * kMaxP));
  st.ctrl_max = s0;
  bool fin = std::isfinite(st.max_dP) && std::isfinite(st.nres_max) && std::isfinite(s0);
  double jmax = 0.0;
  for (int r = 0; r < h.p; ++r) {
    double jr = 0.0;
    for (int a = 0; a < 3; ++a) {
      if (!h.ax[a].active || h.ax[a].B < 2) continue;
      const double raw_j = val(kSlotJ + a * kMaxP + r);
      const double sr = std::max(val(kSlotS + a * kMaxP + r), s0);
      if (!std::isfinite(raw_j)) fin = false;
      jr = std::max(jr, sr > 0.0 ? raw_j / sr : 0.0);
    }
    st.jump[r] = jr;
    jmax = std::max(jmax, jr);
  }
  st.converged = (jump_tol > 0.0 && jmax < jump_tol) ? 1 : 0;
  if (out) *out = st;
  *finite = fin;
  return MFA_OK;
}

// A handle is usable unless it lives in the no-allocation array of its
// device and a newer no-allocation handle has taken that array since.
mfa_status check_handle(const mfa_handle *H) {
  if (!H) return fail(MFA_EINVAL, "null handle");
  if (H->h.noalloc_gen != 0 && noalloc_current(H->h.device) != H->h.noalloc_gen)
    return fail(MFA_EINVAL,
                "the device's no-allocation array now holds a newer handle (mfa_create_noalloc)");
  return MFA_OK;
}

}  // namespace

extern "C" {

const char *mfa_last_error(void) { return g_last_error.c_str(); }

mfa_status mfa_workspace_size(const mfa_problem *prob, size_t *bytes) {
  if (!prob || !bytes) return fail(MFA_EINVAL, "null pointer");
  Handle tmp;
  std::string msg = plan_problem(*prob, &tmp);
  if (!msg.empty()) return fail(MFA_EINVAL, msg);
  *bytes = layout_workspace(&tmp, nullptr);
  return MFA_OK;
}

}  // extern "C"

namespace {

// Plan, lay out the workspace at `workspace` and run the setup chains.
// `serial` keeps every launch on the caller's stream (no auxiliary streams,
// no autotuning timers): the no-allocation entry point creates no HIP
// objects.
mfa_status create_handle(const mfa_problem *prob, void *workspace, size_t bytes, void *hip_stream,
                         bool serial, uint64_t noalloc_gen, mfa_handle **out) {
  mfa_handle *H = new (std::nothrow) mfa_handle();
  if (!H) return fail(MFA_ENOMEM, "host allocation failed");
  Handle &h = H->h;
  std::string msg = plan_problem(*prob, &h);
  if (!msg.empty()) {
    delete H;
    return fail(MFA_EINVAL, msg);
  }
  const size_t need = layout_workspace(&h, nullptr);
  if (bytes < need) {
    delete H;
    return fail(MFA_ENOMEM, "workspace smaller than mfa_workspace_size");
  }
  h.ws = (char *)workspace;
  h.ws_bytes = bytes;
  h.serial = serial;
  h.noalloc_gen = noalloc_gen;
  // diagnostic: MFA_UNFUSED_CORRECTION=1 runs the split-BF16 correction as
  // three separate passes (the same arithmetic) instead of the fused one
  {
    const char *env = getenv("MFA_UNFUSED_CORRECTION");
    h.fuse21 = !(env && env[0] == '1');
  }
  layout_workspace(&h, h.ws);
  h.stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&h.device);
  if (e != hipSuccess) {
    delete H;
    return hip_fail(e, "hipGetDevice");
  }
  auto bail = [&](hipError_t err, const char *where) {
    // work already queued may still read the plan image or the workspace
    (void)hipStreamSynchronize(h.stream);
    delete H;
    return hip_fail(err, where);
  };
  if ((e = launch_zero_slots(h.stream, (unsigned long long *)h.flag, 2)) != hipSuccess)
    return bail(e, "zero flag");
  if ((e = launch_fill(h.stream, h.P, h.nctrl_total, 0.0)) != hipSuccess) return bail(e, "fill P");
  h.p_zero = true;
  // the plan image stays alive until the synchronisation at the end of setup
  std::vector<char> plan_img;
  if ((e = upload_plan(&h, plan_img)) != hipSuccess) return bail(e, "upload plan");
  // Setup (basis, Gram, batched Cholesky, inverses, operator tables) runs
  // stage by stage, each stage of every active axis in one launch on the
  // caller's stream; the variants' tables follow per axis.
  if (h.variant != MFA_VARIANT_CLAMPED && (e = setup_axes(&h, h.stream)) != hipSuccess)
    return bail(e, "setup");
  if (h.precision == MFA_PREC_MIXED_BF16 && (e = setup_mfma_axes(&h, h.stream)) != hipSuccess)
    return bail(e, "setup");
  if (h.variant != MFA_VARIANT_SCHWARZ)
    for (int a = 0; a < 3; ++a)
      if (h.ax[a].active && (e = setup_variant_axis(&h, a, h.stream)) != hipSuccess) return bail(e, "setup");
  // the pivot flag (an int in the first of two zeroed 8-byte slots): through
  // this thread's pinned block unless the handle may not allocate
  int flag = 0;
  if (double *pin = noalloc_gen ? nullptr : pinned_block(h.device)) {
    if ((e = launch_pack_slots(h.stream, (const unsigned long long *)h.flag, 1, 1, nullptr, pin)) !=
        hipSuccess)
      return bail(e, "read flag");
    if ((e = hipStreamSynchronize(h.stream)) != hipSuccess) return bail(e, "setup sync");
    unsigned long long bits = 0ull;   // compare bits: the pattern is a denormal
    std::memcpy(&bits, pin, sizeof(bits));
    flag = bits != 0ull;
  } else {
    if ((e = hipMemcpyAsync(&flag, h.flag, sizeof(int), hipMemcpyDeviceToHost, h.stream)) != hipSuccess)
      return bail(e, "read flag");
    if ((e = hipStreamSynchronize(h.stream)) != hipSuccess) return bail(e, "setup sync");
  }
  if (flag) {
    delete H;
    return fail(MFA_ESINGULAR,
                "a local normal matrix is not positive definite (a basis function without data)");
  }
  *out = H;
  return MFA_OK;
}

}  // namespace

extern "C" {

mfa_status mfa_ctrl_dims(const mfa_problem *prob, int64_t dims[3]) {
  if (!prob || !dims) return fail(MFA_EINVAL, "null pointer");
  Handle tmp;
  std::string msg = plan_problem(*prob, &tmp);
  if (!msg.empty()) return fail(MFA_EINVAL, msg);
  for (int a = 0; a < 3; ++a) dims[a] = a < tmp.dim ? tmp.ax[a + 3 - tmp.dim].nv : 0;
  return MFA_OK;
}

mfa_status mfa_create(const mfa_problem *prob, void *workspace, size_t bytes, void *hip_stream,
                      mfa_handle **out) {
  if (!prob || !out) return fail(MFA_EINVAL, "null pointer");
  *out = nullptr;
  if (!workspace) return fail(MFA_EINVAL, "null workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(MFA_EINVAL, "workspace not 256-byte aligned");
  return create_handle(prob, workspace, bytes, hip_stream, false, 0, out);
}

mfa_status mfa_create_noalloc(const mfa_problem *prob, void *hip_stream, mfa_handle **out) {
  if (!prob || !out) return fail(MFA_EINVAL, "null pointer");
  *out = nullptr;
  size_t need = 0;
  {
    Handle tmp;
    std::string msg = plan_problem(*prob, &tmp);
    if (!msg.empty()) return fail(MFA_EINVAL, msg);
    need = layout_workspace(&tmp, nullptr);
  }
  if (need > (size_t)MFA_NOALLOC_MAX_BYTES)
    return fail(MFA_ENOMEM, "problem needs " + std::to_string(need) +
                                " bytes of workspace, more than the no-allocation array's " +
                                std::to_string((size_t)MFA_NOALLOC_MAX_BYTES));
  void *ptr = nullptr;
  uint64_t gen = 0;
  hipError_t e = noalloc_scratch(&ptr, &gen);
  if (e != hipSuccess) return hip_fail(e, "no-allocation array (hipGetSymbolAddress)");
  return create_handle(prob, ptr, (size_t)MFA_NOALLOC_MAX_BYTES, hip_stream, true, gen, out);
}

void mfa_destroy(mfa_handle *h) { delete h; }

mfa_status mfa_set_timing(mfa_handle *H, int32_t class_mask) {
  if (mfa_status s0 = check_handle(H)) return s0;
  Handle &h = H->h;
  // events still recorded on the stream return to the pool only once it is idle
  bool pending = false;
  for (auto &v : h.ev_used) pending = pending || !v.empty();
  if (pending) HIP_CHECK(hipStreamSynchronize(h.stream), "set_timing");
  for (auto &v : h.ev_used) {
    for (auto &pr : v) {
      h.ev_pool.push_back(pr.first);
      h.ev_pool.push_back(pr.second);
    }
    v.clear();
  }
  h.timing = class_mask & MFA_K_ALL;
  for (auto &n : h.timing_seen) n = 0;
  return MFA_OK;
}

mfa_status mfa_set_timing_every(mfa_handle *H, int32_t every, int32_t first) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (every < 1 || first < 0 || first >= every)
    return fail(MFA_EINVAL, "timing sample: need every >= 1 and 0 <= first < every");
  Handle &h = H->h;
  h.timing_every = every;
  h.timing_first = first;
  for (auto &n : h.timing_seen) n = 0;
  return MFA_OK;
}

mfa_status mfa_kernel_time(mfa_handle *H, int32_t kclass, double *total_ms, int64_t *launches) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (!total_ms || !launches) return fail(MFA_EINVAL, "null pointer");
  if (kclass < 0 || kclass >= MFA_K_COUNT) return fail(MFA_EINVAL, "kernel class out of range");
  Handle &h = H->h;
  HIP_CHECK(hipStreamSynchronize(h.stream), "kernel_time");
  double tot = 0.0;
  for (auto &pr : h.ev_used[kclass]) {
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, pr.first, pr.second), "kernel_time");
    tot += ms;
    h.ev_pool.push_back(pr.first);
    h.ev_pool.push_back(pr.second);
  }
  *launches = (int64_t)h.ev_used[kclass].size();
  h.ev_used[kclass].clear();
  *total_ms = tot;
  return MFA_OK;
}

static mfa_status load_q(Handle &h, const void *q, mfa_dtype dt) {
  if (dt != MFA_F32 && dt != MFA_F64) return fail(MFA_EINVAL, "bad dtype");
  h.q = q;
  h.q_dtype = dt;
  if (h.rhs == MFA_RHS_DATABOX || h.variant) {   // the data are read by every sweep / the fit
    h.have_rhs = true;
    return MFA_OK;
  }
  hipError_t e = dt == MFA_F32 ? project<float>(h, (const float *)q) : project<double>(h, (const double *)q);
  if (e != hipSuccess) return hip_fail(e, "project");
  h.have_rhs = true;
  return MFA_OK;
}

// Whether a NORMAL-mode sweep starts with the residual stencil kernel (the
// conditions of sweep_normal's first two branches).
static bool sweep_uses_resid_kernel(const Handle &h) {
  if (h.rhs == MFA_RHS_DATABOX) return false;
  if (h.precision == MFA_PREC_MIXED_BF16 && mfma_ok(h)) return true;
  return fast_sweep_ok(h, h.precision != MFA_PREC_FP64 ? sizeof(float) : sizeof(double));
}

static mfa_status do_sweep(Handle &h, bool metrics) {
  // Reduction slots: sweep k (0-based h.sweep) writes set k % 2, which is
  // zero when it starts.  The residual kernel of sweep k records the max
  // |correction| of sweep k-1 (set (k+1) % 2) into the history and clears
  // that set for sweep k+1; the host reads a sweep's set only right after it
  // (stream-synchronised), before the next sweep is queued.  Sweeps without
  // the residual kernel clear their own set with one small launch.
  const int64_t nset = (int64_t)kNumSlots * kSlotCopies;
  unsigned long long *cur = h.slot_base + (h.sweep & 1) * nset;
  unsigned long long *prev = h.slot_base + ((h.sweep + 1) & 1) * nset;
  h.slots = cur;
  double *hist = h.sweep >= 1 ? h.hist : nullptr;
  const int hidx = (h.sweep - 1 + kHist) % kHist;
  SlotTurn turn;
  hipError_t e = hipSuccess;
  // P = 0 is known only for the first sweep of a cold-start encode
  const bool p_zero = h.p_known_zero && h.sweep == 0;
  h.p_known_zero = false;
  if (sweep_uses_resid_kernel(h)) {
    // the first sweep also clears its own set (both sets start cleared)
    if (h.sweep == 0 && (e = launch_zero_slots(h.stream, h.slot_base, 2 * (int)nset)) != hipSuccess)
      return hip_fail(e, "zero slots");
    turn = SlotTurn{prev, hist, hidx};
  } else {
    e = launch_zero_slots(h.stream, cur, (int)nset, hist, hidx, prev);
    if (e != hipSuccess) return hip_fail(e, "zero slots");
  }
  if (h.rhs == MFA_RHS_DATABOX) {
    e = sweep_databox(h, metrics);
    if (e != hipSuccess) return hip_fail(e, "sweep");
    if (metrics) {
      TimeScope ts(h, MFA_K_METRICS);
      e = launch_deriv_scale(h);
      if (e != hipSuccess) return hip_fail(e, "metrics");
    }
  } else {
    e = sweep_normal(h, turn, p_zero);
    if (e != hipSuccess) return hip_fail(e, "sweep");
    if (metrics) {
      e = sweep_metrics(h);
      if (e != hipSuccess) return hip_fail(e, "metrics");
    }
  }
  h.sweep++;
  return MFA_OK;
}

mfa_status mfa_schwarz_step(mfa_handle *H, const void *q_dev, mfa_dtype q_dtype, mfa_step_stats *out) {
  if (mfa_status s0 = check_handle(H)) return s0;
  Handle &h = H->h;
  hipSetDevice(h.device);
  h.p_zero = false;
  if (q_dev) {
    mfa_status s = load_q(h, q_dev, q_dtype);
    if (s != MFA_OK) return s;
  } else if (!h.have_rhs) {
    return fail(MFA_EINVAL, "no data loaded: pass q_dev");
  }
  if (h.variant) {
    mfa_status sv = encode_variant(h, out);
    if (sv == MFA_OK && out) sv = residual_stats(h, &out->res_max, &out->res_l2);
    return sv;
  }
  mfa_status s = do_sweep(h, true);
  if (s != MFA_OK) return s;
  bool finite = true;
  s = read_stats(h, out, 0.0, &finite);
  if (s != MFA_OK) return s;
  if (!finite) return fail(MFA_ENOTCONV, "non-finite value in the sweep");
  if (out && (s = residual_stats(h, &out->res_max, &out->res_l2)) != MFA_OK) return s;
  return MFA_OK;
}

mfa_status mfa_encode(mfa_handle *H, const void *q_dev, mfa_dtype q_dtype, int32_t max_sweeps,
                      double jump_tol, int32_t check_every, mfa_step_stats *last) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (!q_dev) return fail(MFA_EINVAL, "null data pointer");
  if (max_sweeps < 1) return fail(MFA_EINVAL, "max_sweeps must be >= 1");
  Handle &h = H->h;
  hipSetDevice(h.device);
  // a cold start needs P = 0, which a new handle already holds
  const bool p_zero = h.p_zero;
  h.p_zero = false;
  mfa_status s = load_q(h, q_dev, q_dtype);
  if (s != MFA_OK) return s;
  if (h.variant) {   // one-shot fit, no sweeps
    h.warm = false;
    return encode_variant(h, last);
  }
  h.sweep = 0;
  if (!h.warm && !p_zero) {
    hipError_t e = launch_fill(h.stream, h.P, h.nctrl_total, 0.0);
    if (e != hipSuccess) return hip_fail(e, "fill P");
  }
  h.p_known_zero = !h.warm;
  h.warm = false;
  mfa_step_stats st{};
  bool converged = false;
  // Check schedule: a fixed stride, or (check_every <= 0) predicted.  Past
  // the first sweeps' transient the jumps decay at the same geometric rate
  // as max |correction|, which every sweep reduces anyway (recorded in
  // h.hist): a check at sweep k with largest jump J predicts the crossing of
  // the tolerance after log(tol / J) / log(rate) more sweeps, the rate taken
  // from the corrections of sweeps k-2 .. k.  The first check comes at sweep
  // 6, after the transient.
  //
  // The count is rounded up, except for the prediction made at the first
  // check when an axis has four or more subdomains: there the contraction
  // is still speeding up at sweep 6 (a correction crosses one subdomain per
  // sweep, so the slowest error components take longer to form), the rate
  // from sweeps 4..6 is slower than the one that follows, and the count is
  // rounded down.  With at most two subdomains per axis the rate is steady
  // by then and the rounded-up count is the crossing itself.
  int bmax = 1;
  for (int a = 0; a < 3; ++a)
    if (h.ax[a].active) bmax = std::max(bmax, h.ax[a].B);
  bool first_prediction = true;
  int next_check = jump_tol > 0.0 ? (check_every > 0 ? check_every : 6) : max_sweeps;
  for (int k = 1; k <= max_sweeps; ++k) {
    const bool check = k == next_check || k == max_sweeps;
    s = do_sweep(h, check);
    if (s != MFA_OK) return s;
    if (!check) continue;
    bool finite = true;
    // the predicted schedule also needs max |correction| of sweep k - 2
    const bool want_hist = jump_tol > 0.0 && check_every <= 0 && k >= 3;
    double d2 = 0.0;
    s = read_stats(h, &st, jump_tol, &finite, want_hist ? &d2 : nullptr, (k - 3 + kHist) % kHist);
    if (s != MFA_OK) return s;
    if (!finite) {
      if (last) *last = st;
      return fail(MFA_ENOTCONV, "non-finite value in the sweep");
    }
    if (st.converged) {
      converged = true;
      break;
    }
    if (check_every > 0) {
      next_check = k + check_every;
    } else {
      double jm = 0.0;
      for (int r = 0; r < h.p; ++r) jm = std::max(jm, st.jump[r]);
      int stride = 4;
      if (k >= 3) {
        const double d0 = st.max_dP;
        if (d2 > 0.0 && d0 > 0.0 && d0 < d2 && jm > 0.0) {
          const double rate = std::sqrt(d0 / d2);
          const double need = std::log(jump_tol / jm) / std::log(rate);
          const double n = first_prediction && bmax >= 4 ? std::floor(need) : std::ceil(need);
          stride = (int)std::min(32.0, std::max(1.0, n));
        }
      }
      first_prediction = false;
      next_check = k + stride;
    }
  }
  if (last) *last = st;
  if (jump_tol > 0.0 && !converged) return fail(MFA_ENOTCONV, "jump tolerance not reached");
  return MFA_OK;
}

mfa_status mfa_fit_error(mfa_handle *H, double *res_max, double *res_l2) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (!res_max || !res_l2) return fail(MFA_EINVAL, "null pointer");
  Handle &h = H->h;
  hipSetDevice(h.device);
  if (!h.q) return fail(MFA_EINVAL, "no data loaded: run mfa_encode or mfa_schwarz_step first");
  return residual_stats(h, res_max, res_l2);
}

mfa_status mfa_decode(mfa_handle *H, void *out_dev, mfa_dtype out_dtype, const int32_t *deriv) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (!out_dev) return fail(MFA_EINVAL, "null output pointer");
  Handle &h = H->h;
  hipSetDevice(h.device);
  std::vector<Step> st;
  for (int a = 2; a >= 0; --a) {
    if (!h.ax[a].active) continue;
    int r = 0;
    if (deriv) r = deriv[a - (3 - h.dim)];
    if (r < 0 || r > h.p) return fail(MFA_EINVAL, "derivative order out of range");
    st.push_back({a, h.variant ? &h.ax[a].Nv[r] : &h.ax[a].N[r]});
  }
  hipError_t e;
  TimeScope ts(h, MFA_K_DECODE);
  if (out_dtype != MFA_F32 && out_dtype != MFA_F64) return fail(MFA_EINVAL, "bad dtype");
  if (grid_pass_ok(h) && !h.variant) {
    int r[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
      if (h.ax[a].active && deriv) r[a] = deriv[a - (3 - h.dim)];
    e = launch_decode_grid(h, out_dev, out_dtype == MFA_F32, r);
    if (e == hipSuccess) return MFA_OK;
    if (e != hipErrorNotSupported) return hip_fail(e, "decode");
  }
  if (out_dtype == MFA_F32)
    e = run_chain<double, float>(h, h.P, model_dims(h), st, (float *)out_dev, EPI_STORE, nullptr, 0,
                                 nullptr, 0, h.s1, h.s2);
  else if (out_dtype == MFA_F64)
    e = run_chain<double, double>(h, h.P, model_dims(h), st, (double *)out_dev, EPI_STORE, nullptr, 0,
                                  nullptr, 0, h.s1, h.s2);
  else
    return fail(MFA_EINVAL, "bad dtype");
  if (e != hipSuccess) return hip_fail(e, "decode");
  return MFA_OK;
}

mfa_status mfa_decode_points(mfa_handle *H, const double *u_dev, int64_t npoints, void *out_dev,
                             mfa_dtype out_dtype, const int32_t *deriv) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (npoints < 0) return fail(MFA_EINVAL, "negative point count");
  if (npoints > 0 && (!u_dev || !out_dev)) return fail(MFA_EINVAL, "null pointer");
  if (out_dtype != MFA_F32 && out_dtype != MFA_F64) return fail(MFA_EINVAL, "bad dtype");
  Handle &h = H->h;
  if (h.variant) return fail(MFA_EINVAL, "decode at points is for the Schwarz model only");
  hipSetDevice(h.device);
  int r[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    if (!h.ax[a].active || !deriv) continue;
    r[a] = deriv[a - (3 - h.dim)];
    if (r[a] < 0 || r[a] > h.p) return fail(MFA_EINVAL, "derivative order out of range");
  }
  TimeScope ts(h, MFA_K_DECODE);
  hipError_t e = launch_decode_points(h, u_dev, npoints, out_dev, out_dtype == MFA_F32, r);
  if (e != hipSuccess) return hip_fail(e, "decode points");
  return MFA_OK;
}

mfa_status mfa_get_ctrl(mfa_handle *H, double *ctrl, int32_t on_device) {
  if (mfa_status s0 = check_handle(H)) return s0;
  if (!ctrl) return fail(MFA_EINVAL, "null pointer");
  Handle &h = H->h;
  hipSetDevice(h.device);
  const size_t bytes = sizeof(double) * (size_t)h.nctrl_total;
  HIP_CHECK(hipMemcpyAsync(ctrl, h.P, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           h.stream),
            "get_ctrl");
  if (!on_device) HIP_CHECK(hipStreamSynchronize(h.stream), "get_ctrl");
  return MFA_OK;
}

mfa_status mfa_set_stream(mfa_handle *H, void *hip_stream) {
  if (mfa_status s0 = check_handle(H)) return s0;
  Handle &h = H->h;
  hipSetDevice(h.device);
  // everything queued so far on the old stream completes first
  HIP_CHECK(hipStreamSynchronize(h.stream), "set_stream");
  h.stream = (hipStream_t)hip_stream;
  return MFA_OK;
}

mfa_status mfa_set_ctrl(mfa_handle *H, const double *ctrl, int32_t on_device) {
  if (mfa_status s0 = check_handle(H)) return s0;
  Handle &h = H->h;
  hipSetDevice(h.device);
  if (!ctrl) {   // warm start from the control points the handle holds
    h.warm = true;
    return MFA_OK;
  }
  const size_t bytes = sizeof(double) * (size_t)h.nctrl_total;
  h.p_zero = false;
  HIP_CHECK(hipMemcpyAsync(h.P, ctrl, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           h.stream),
            "set_ctrl");
  if (!on_device) HIP_CHECK(hipStreamSynchronize(h.stream), "set_ctrl");
  h.warm = true;
  return MFA_OK;
}

mfa_status mfa_inspect(mfa_handle *H, int32_t table, int32_t axis, int32_t block, double *host_out,
                       size_t count, size_t *needed) {
  if (mfa_status s0 = check_handle(H)) return s0;
  Handle &h = H->h;
  if (h.variant == MFA_VARIANT_CLAMPED) return fail(MFA_EINVAL, "no such table for the clamped variant");
  hipSetDevice(h.device);
  if (table != MFA_T_RHS && (axis < 0 || axis >= h.dim)) return fail(MFA_EINVAL, "axis out of range");
  const Axis &X = h.ax[table == MFA_T_RHS ? 0 : axis + 3 - h.dim];
  if ((table == MFA_T_CHOL || table == MFA_T_INV) && (block < 0 || block >= X.B))
    return fail(MFA_EINVAL, "block out of range");
  const int p = h.p;
  std::vector<double> buf;
  switch (table) {
    case MFA_T_BASIS: {
      buf.resize((size_t)X.m * (p + 1));
      HIP_CHECK(hipMemcpyAsync(buf.data(), X.N[0].val, sizeof(double) * buf.size(), hipMemcpyDeviceToHost,
                               h.stream), "inspect");
      break;
    }
    case MFA_T_SPAN: {
      std::vector<int> s(X.m);
      HIP_CHECK(hipMemcpyAsync(s.data(), X.d_span, sizeof(int) * s.size(), hipMemcpyDeviceToHost, h.stream),
                "inspect");
      HIP_CHECK(hipStreamSynchronize(h.stream), "inspect");
      buf.assign(s.begin(), s.end());
      break;
    }
    case MFA_T_GRAM: {
      buf.resize((size_t)(p + 1) * X.n);
      HIP_CHECK(hipMemcpyAsync(buf.data(), X.d_gram, sizeof(double) * buf.size(), hipMemcpyDeviceToHost,
                               h.stream), "inspect");
      break;
    }
    case MFA_T_CHOL: {
      const int64_t F = X.blk[block].F1 - X.blk[block].F0;
      buf.resize((size_t)(p + 1) * F);
      HIP_CHECK(hipMemcpyAsync(buf.data(), X.d_chol + X.chol_off[block], sizeof(double) * buf.size(),
                               hipMemcpyDeviceToHost, h.stream), "inspect");
      break;
    }
    case MFA_T_INV: {
      const int64_t F = X.blk[block].F1 - X.blk[block].F0;
      buf.resize((size_t)F * F);
      HIP_CHECK(hipMemcpyAsync(buf.data(), X.d_inv + X.inv_off[block], sizeof(double) * buf.size(),
                               hipMemcpyDeviceToHost, h.stream), "inspect");
      break;
    }
    case MFA_T_RHS: {
      if (!h.have_rhs || h.rhs != MFA_RHS_NORMAL) return fail(MFA_EINVAL, "no N^T Q (NORMAL mode only)");
      buf.resize((size_t)h.nctrl_total);
      HIP_CHECK(hipMemcpyAsync(buf.data(), h.c, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, h.stream),
                "inspect");
      break;
    }
    default:
      return fail(MFA_EINVAL, "unknown table");
  }
  HIP_CHECK(hipStreamSynchronize(h.stream), "inspect");
  if (needed) *needed = buf.size();
  if (host_out) {
    if (count < buf.size()) return fail(MFA_EINVAL, "output buffer too small");
    std::memcpy(host_out, buf.data(), sizeof(double) * buf.size());
  }
  return MFA_OK;
}

}  // extern "C"
