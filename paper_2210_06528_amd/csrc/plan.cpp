// Host planner: validates a problem, computes the subdomain index ranges of
// Section 2.2 with exact integer arithmetic, and lays out the workspace.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "mfa_internal.hpp"

namespace mfa {

namespace {

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Right-continuous span of data point i: the largest s with t_s <= u_i,
// clamped to [p, n-1], for u_i = i/(m-1) and t_j = (j-p)/(n-p).
inline int span_of(int64_t i, int64_t m, int n, int p) {
  int64_t s = p + (i * (n - p)) / (m - 1);
  return (int)std::min<int64_t>(s, n - 1);
}

// smallest data index whose span is >= s
inline int64_t first_with_span_ge(int s, int64_t m, int n, int p) {
  if (s <= p) return 0;
  return ceil_div((int64_t)(s - p) * (m - 1), n - p);
}

// largest data index whose span is <= s
inline int64_t last_with_span_le(int s, int64_t m, int n, int p) {
  if (s >= n - 1) return m - 1;
  return ceil_div((int64_t)(s - p + 1) * (m - 1), n - p) - 1;
}

// p * (n-p) * (Greville abscissa xi_k): the sum of knots t_{k+1..k+p} scaled
// to integers.
inline int64_t greville_num(int k, int n, int p) {
  int64_t s = 0;
  for (int j = k + 1; j <= k + p; ++j) s += std::min(std::max(j - p, 0), n - p);
  return s;
}

}  // namespace

std::string plan_problem(const mfa_problem &prob, Handle *h) {
  std::ostringstream err;
  if (prob.dim < 1 || prob.dim > 3) return "dim must be 1, 2 or 3";
  const int p = prob.degree;
  if (p < 1 || p > kMaxP) {
    err << "degree must be in 1.." << kMaxP;
    return err.str();
  }
  if (prob.overlap < 0) return "overlap must be >= 0";
  if (prob.precision < 0 || prob.precision > 2) return "precision out of range";
  if (prob.combine < 0 || prob.combine > 1) return "combine out of range";
  if (prob.rhs < 0 || prob.rhs > 1) return "rhs out of range";
  if (prob.variant < 0 || prob.variant > 2) return "variant out of range";
  if (prob.variant != MFA_VARIANT_SCHWARZ &&
      (prob.precision != MFA_PREC_FP64 || prob.rhs != MFA_RHS_NORMAL))
    return "the decoupled and clamped variants take precision FP64 and rhs NORMAL";
  h->prob = prob;
  h->dim = prob.dim;
  h->p = p;
  h->overlap = prob.overlap;
  h->precision = prob.precision;
  h->combine = prob.combine;
  h->rhs = prob.rhs;
  h->variant = prob.variant;
  const int o = prob.overlap;
  const int minov = std::max(1, p / 2);
  h->nctrl_total = 1;
  h->npts_total = 1;
  for (int ia = 0; ia < 3; ++ia) h->ax[ia] = Axis();
  for (int a = 0; a < prob.dim; ++a) {
    Axis &X = h->ax[a + 3 - prob.dim];
    X.active = true;
    X.m = prob.npts[a];
    X.B = prob.nsub[a];
    if (X.B < 1) return "nsub must be >= 1";
    if (prob.nctrl[a] == nullptr) return "nctrl pointer is null";
    int n = 0;
    for (int b = 0; b < X.B; ++b) {
      if (prob.nctrl[a][b] < 1) return "owned control count must be >= 1";
      n += prob.nctrl[a][b];
    }
    X.n = n;
    {
      const double lo = prob.lo[a], hi = prob.hi[a];
      if (!std::isfinite(lo) || !std::isfinite(hi)) return "axis extent lo/hi not finite";
      if (hi < lo) return "axis extent with hi < lo";
      X.dscale = hi > lo ? 1.0 / (hi - lo) : 1.0;
    }
    if (prob.weights[a]) {
      X.w.assign(prob.weights[a], prob.weights[a] + n);
      for (double v : X.w)
        if (!std::isfinite(v) || !(v > 0.0)) return "a weight is not positive and finite";
    }
    if (prob.variant == MFA_VARIANT_CLAMPED) {
      // own clamped knots per block; neighbours share the interface control
      // point; interface b sits on the data point nearest to (m-1) x (spans
      // before it) / (all spans), halves rounded up
      if (!X.w.empty()) return "the clamped variant takes no weights";
      if (X.m < 2) return "fewer than 2 data points on an axis";
      int64_t tot = 0;
      for (int b = 0; b < X.B; ++b) {
        if (prob.nctrl[a][b] < p + 1) return "a clamped block needs at least p+1 control points";
        tot += prob.nctrl[a][b] - p;
      }
      X.ccut.assign(X.B + 1, 0);
      X.coff.assign(X.B, 0);
      X.csz.assign(X.B, 0);
      int64_t acc = 0;
      for (int b = 0; b + 1 < X.B; ++b) {
        acc += prob.nctrl[a][b] - p;
        X.ccut[b + 1] = (int)(((X.m - 1) * acc * 2 + tot) / (2 * tot));
      }
      X.ccut[X.B] = (int)(X.m - 1);
      X.LLv = 0;
      for (int b = 0; b < X.B; ++b) {
        X.csz[b] = prob.nctrl[a][b];
        X.coff[b] = b == 0 ? 0 : X.coff[b - 1] + X.csz[b - 1] - 1;
        const int64_t nd = (int64_t)X.ccut[b + 1] - X.ccut[b] + 1;
        if (nd < X.csz[b]) return "a clamped block has fewer data points than control points";
        X.LLv = std::max(X.LLv, nd);
      }
      X.nv = n - (X.B - 1);
      X.n = X.nv;
      h->nctrl_total *= X.nv;
      h->npts_total *= X.m;
      continue;
    }
    if (n < p + 1) return "fewer than p+1 control points on an axis";
    if (X.m < 2) return "fewer than 2 data points on an axis";
    if (X.m < n) return "fewer data points than control points on an axis";
    if (X.B > 1) {
      if (o < minov) {
        err << "overlap " << o << " below max(1, floor(p/2)) = " << minov;
        return err.str();
      }
      for (int b = 0; b < X.B; ++b)
        if (prob.nctrl[a][b] < std::max(p + 1, 2 * o)) {
          err << "owned block of " << prob.nctrl[a][b] << " control points below max(p+1, 2*overlap)";
          return err.str();
        }
    }
    const int64_t m = X.m;
    // interfaces: Greville midpoint between the last owned control point of
    // block b and the first of block b+1, as the exact fraction num/den
    const int64_t den = 2LL * p * (n - p);
    std::vector<int64_t> cuts(X.B + 1, 0);
    cuts[X.B] = m;
    X.ustar.assign(std::max(0, X.B - 1), 0.0);
    X.span_if.assign(std::max(0, X.B - 1), 0);
    int c = 0;
    for (int b = 0; b + 1 < X.B; ++b) {
      c += prob.nctrl[a][b];
      const int64_t num = greville_num(c - 1, n, p) + greville_num(c, n, p);
      cuts[b + 1] = ceil_div(num * (m - 1), den);
      const double us = (double)num / (double)den;
      X.ustar[b] = us;
      // right-continuous span of u* = num/den: s - p = floor(num (n-p) / den)
      const int64_t s = p + (num * (int64_t)(n - p)) / den;
      X.span_if[b] = (int)std::min<int64_t>(s, n - 1);
    }
    X.blk.resize(X.B);
    int c0 = 0;
    X.Fmax = 0;
    for (int b = 0; b < X.B; ++b) {
      Block &B = X.blk[b];
      B.c0 = c0;
      B.c1 = c0 + prob.nctrl[a][b];
      B.F0 = b > 0 ? std::max(0, B.c0 - o) : 0;
      B.F1 = b < X.B - 1 ? std::min(n, B.c1 + o) : n;
      B.E0 = std::max(0, B.F0 - p);
      B.E1 = std::min(n, B.F1 + p);
      const int smin = std::max(p, B.F0);
      const int smax = std::min(n - 1, B.F1 - 1 + p);
      B.D0 = first_with_span_ge(smin, m, n, p);
      B.D1 = last_with_span_le(smax, m, n, p) + 1;
      B.own0 = cuts[b];
      B.own1 = cuts[b + 1];
      if (B.own1 <= B.own0) return "a subdomain owns no data point";
      X.Fmax = std::max<int64_t>(X.Fmax, B.F1 - B.F0);
      c0 = B.c1;
    }
    X.ns.assign(n, 0);
    X.blo.assign(n, X.B);
    X.bhi.assign(n, -1);
    X.owner.assign(n, 0);
    for (int b = 0; b < X.B; ++b) {
      for (int k = X.blk[b].F0; k < X.blk[b].F1; ++k) {
        X.ns[k]++;
        X.blo[k] = std::min(X.blo[k], b);
        X.bhi[k] = std::max(X.bhi[k], b);
      }
      for (int k = X.blk[b].c0; k < X.blk[b].c1; ++k) X.owner[k] = b;
    }
    X.pown.assign(m, 0);
    for (int b = 0; b < X.B; ++b)
      for (int64_t i = X.blk[b].own0; i < X.blk[b].own1; ++i) X.pown[i] = b;
    // table widths
    X.LNT = 0;
    for (int k = 0; k < n; ++k) {
      const int64_t lo = first_with_span_ge(std::max(k, p), m, n, p);
      const int64_t hi = last_with_span_le(std::min(k + p, n - 1), m, n, p);
      X.LNT = std::max<int64_t>(X.LNT, hi - lo + 1);
    }
    X.LM = 0;
    for (int k = 0; k < n; ++k) {
      int64_t len;
      if (prob.combine == MFA_COMBINE_AVG)
        len = X.blk[X.bhi[k]].F1 - X.blk[X.blo[k]].F0;
      else
        len = X.blk[X.owner[k]].F1 - X.blk[X.owner[k]].F0;
      X.LM = std::max(X.LM, len);
    }
    X.LOm = X.Fmax;
    X.LJ = 0;
    for (int b = 0; b + 1 < X.B; ++b)
      X.LJ = std::max<int64_t>(X.LJ, X.blk[b + 1].F1 - X.blk[b].F0);
    X.ND = 0;
    for (int r = 0; r < p; ++r) X.ND += n - r;
    X.chol_off.resize(X.B);
    X.inv_off.resize(X.B);
    X.chol_total = X.inv_total = 0;
    for (int b = 0; b < X.B; ++b) {
      const int64_t F = X.blk[b].F1 - X.blk[b].F0;
      X.chol_off[b] = X.chol_total;
      X.inv_off[b] = X.inv_total;
      X.chol_total += (p + 1) * F;
      X.inv_total += F * F;
    }
    // segmented (DATABOX) layouts
    X.doff.resize(X.B + 1);
    X.foff.resize(X.B + 1);
    X.SD = X.SF = 0;
    X.LNsT = 0;
    for (int b = 0; b < X.B; ++b) {
      X.doff[b] = X.SD;
      X.foff[b] = X.SF;
      X.SD += X.blk[b].D1 - X.blk[b].D0;
      X.SF += X.blk[b].F1 - X.blk[b].F0;
      for (int k = X.blk[b].F0; k < X.blk[b].F1; ++k) {
        int64_t lo = first_with_span_ge(std::max(k, p), m, n, p);
        int64_t hi = last_with_span_le(std::min(k + p, n - 1), m, n, p);
        lo = std::max(lo, X.blk[b].D0);
        hi = std::min(hi, X.blk[b].D1 - 1);
        X.LNsT = std::max<int64_t>(X.LNsT, hi - lo + 1);
      }
    }
    X.doff[X.B] = X.SD;
    X.foff[X.B] = X.SF;
    X.nv = n;
    if (prob.variant == MFA_VARIANT_DECOUPLED) {
      X.nv = (int)X.SF;
      X.LLv = 0;
      for (int b = 0; b < X.B; ++b) X.LLv = std::max<int64_t>(X.LLv, X.blk[b].D1 - X.blk[b].D0);
    }
    h->nctrl_total *= X.nv;
    h->npts_total *= m;
  }
  for (int ia = 0; ia < 3; ++ia)
    if (!h->ax[ia].active) h->ax[ia].nv = 1;
  return "";
}

namespace {

struct Bump {
  char *base;
  size_t off = 0;
  explicit Bump(char *b) : base(b) {}
  template <typename T>
  T *take(int64_t count) {
    off = (off + 255) & ~(size_t)255;
    T *ptr = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    return ptr;
  }
  void ell(Ell &e, int R, int C, int64_t L, bool with_float) {
    e.R = R;
    e.C = C;
    e.L = (int)std::max<int64_t>(L, 1);
    e.len = take<int>(R);
    e.col = take<int>((int64_t)R * e.L);
    e.val = take<double>((int64_t)R * e.L);
    e.valf = with_float ? take<float>((int64_t)R * e.L) : nullptr;
  }
};

}  // namespace

// Largest intermediates of the pass chains between the data grid and a
// control grid with cn[a] control points per axis: the fit / projection chain
// (axis 2 first), the decode chain (axis 2 first) and every jump chain (rows
// along the interface axis, then the data points of the other axes).  A
// chain's last pass writes its output directly.
static void chain_scratch(const Handle *h, const int64_t cn[3], int64_t *s1, int64_t *s2) {
  auto upd = [&](int which, int64_t v) {
    if (which == 0) *s1 = std::max(*s1, v);
    else *s2 = std::max(*s2, v);
  };
  int first = 0;
  while (first < 2 && !h->ax[first].active) ++first;
  Dims d{{h->ax[0].m, h->ax[1].m, h->ax[2].m}};
  int w = 0;
  for (int ia = 2; ia > first; --ia) {
    if (!h->ax[ia].active) continue;
    d.d[ia] = cn[ia];
    upd(w, d.total());
    w ^= 1;
  }
  Dims e{{cn[0], cn[1], cn[2]}};
  w = 0;
  for (int ia = 2; ia > first; --ia) {
    if (!h->ax[ia].active) continue;
    e.d[ia] = h->ax[ia].m;
    upd(w, e.total());
    w ^= 1;
  }
  for (int a = 0; a < 3; ++a) {
    if (!h->ax[a].active || h->ax[a].B < 2) continue;
    Dims j{{cn[0], cn[1], cn[2]}};
    j.d[a] = (int64_t)(h->ax[a].B - 1) * h->p;
    w = 0;
    upd(w, j.total());
    for (int c = 0; c < 3; ++c) {
      if (c == a || !h->ax[c].active) continue;
      w ^= 1;
      j.d[c] = h->ax[c].m;
      upd(w, j.total());
    }
  }
}

// Workspace of the CLAMPED variant: its block tables, fit / decode / jump
// operators, control points and chain scratch only.
static size_t layout_clamped(Handle *h, char *base) {
  Bump bp(base);
  const int p = h->p;
  for (int ia = 0; ia < 3; ++ia) {
    Axis &X = h->ax[ia];
    if (!X.active) continue;
    X.d_ccut = bp.take<int>(X.B + 1);
    X.d_coff = bp.take<int>(X.B);
    X.d_csz = bp.take<int>(X.B);
  }
  h->upload_bytes = bp.off;
  for (int ia = 0; ia < 3; ++ia) {
    Axis &X = h->ax[ia];
    if (!X.active) continue;
    const int nif = X.B - 1;
    bp.ell(X.Lv, X.nv, (int)X.m, X.LLv, false);
    for (int r = 0; r <= p; ++r) bp.ell(X.Nv[r], (int)X.m, X.nv, p + 1, false);
    bp.ell(X.Jv, nif * p, X.nv, 2 * (p + 1), false);
    X.d_gidJ = bp.take<int>((int64_t)nif * p);
  }
  const int64_t NC = h->nctrl_total;
  h->c = bp.take<double>(1);
  h->P = bp.take<double>(NC);
  h->g = bp.take<double>(1);
  const int64_t cn[3] = {h->ax[0].nv, h->ax[1].nv, h->ax[2].nv};
  int64_t s1 = NC, s2 = NC;
  chain_scratch(h, cn, &s1, &s2);
  h->s1 = bp.take<double>(s1);
  h->s2 = bp.take<double>(s2);
  h->s1n = s1;
  h->s2n = s2;
  h->slot_base = bp.take<unsigned long long>(2 * (int64_t)kNumSlots * kSlotCopies);
  h->slots = h->slot_base;
  h->flag = bp.take<int>(4);
  h->hist = bp.take<double>(kHist);
  h->res_slots = bp.take<unsigned long long>(2 * (int64_t)kSlotCopies);
  return bp.off + 256;
}

size_t layout_workspace(Handle *h, char *base) {
  if (h->variant == MFA_VARIANT_CLAMPED) return layout_clamped(h, base);
  Bump bp(base);
  const int p = h->p;
  const bool mixed = h->precision != MFA_PREC_FP64;
  // host-planned tables of every axis first, in one contiguous region that
  // setup uploads with a single copy
  for (int ia = 0; ia < 3; ++ia) {
    Axis &X = h->ax[ia];
    if (!X.active) {
      X.d_acoef = bp.take<double>((int64_t)(2 * p + 1) * X.n);
      continue;
    }
    const int n = X.n;
    const int nif = X.B - 1;
    X.d_choff = bp.take<int>(X.B);
    X.d_foff = bp.take<int>(X.B);
    X.d_blk = bp.take<int>(8LL * X.B);
    X.d_blo = bp.take<int>(n);
    X.d_bhi = bp.take<int>(n);
    X.d_owner = bp.take<int>(n);
    X.d_ns = bp.take<int>(n);
    X.d_pown = bp.take<int>(X.m);
    X.d_ustar = bp.take<double>(nif);
    X.d_span_if = bp.take<int>(nif);
    X.d_w = X.w.empty() ? nullptr : bp.take<double>(n);
  }
  h->upload_bytes = bp.off;
  for (int ia = 0; ia < 3; ++ia) {
    Axis &X = h->ax[ia];
    if (!X.active) continue;
    X.d_acoef = bp.take<double>((int64_t)(2 * p + 1) * X.n);
    X.d_rdiag = bp.take<double>(X.SF);
    const int n = X.n;
    const int64_t m = X.m;
    const int nif = X.B - 1;
    X.d_span = bp.take<int>(m);
    X.d_bas = bp.take<double>(m * (p + 1));
    X.d_gram = bp.take<double>((int64_t)(p + 1) * n);
    X.d_chol = bp.take<double>(X.chol_total);
    X.d_inv = bp.take<double>(X.inv_total);
    X.d_dbas_if = bp.take<double>((int64_t)nif * p * (p + 1));
    X.d_gidJ = bp.take<int>((int64_t)nif * p);
    X.d_gidD = bp.take<int>(X.ND);
    for (int r = 0; r <= p; ++r) bp.ell(X.N[r], (int)m, n, p + 1, false);
    bp.ell(X.NT, n, (int)m, X.LNT, false);
    bp.ell(X.A, n, n, 2 * p + 1, false);
    bp.ell(X.M, n, n, X.LM, mixed);
    if (h->precision == MFA_PREC_MIXED_BF16) {
      X.npad = (n + 31) / 32 * 32 + 32;
      X.d_Mb = bp.take<uint16_t>(2 * (int64_t)((n + 15) / 16 * 16) * X.npad);
      X.d_klo = bp.take<int>((n + 15) / 16);
      X.d_knc = bp.take<int>((n + 15) / 16);
    }
    bp.ell(X.Om, (int)m, n, X.LOm, false);
    X.d_omT = bp.take<double>((int64_t)X.Om.L * m);
    bp.ell(X.J, nif * p, n, X.LJ, false);
    bp.ell(X.D, (int)X.ND, n, p, false);
    if (h->variant == MFA_VARIANT_DECOUPLED) {
      bp.ell(X.Lv, X.nv, (int)m, X.LLv, false);
      for (int r = 0; r <= p; ++r) bp.ell(X.Nv[r], (int)m, X.nv, p + 1, false);
      bp.ell(X.Jv, nif * p, X.nv, 2 * (p + 1), false);
    }
    if (h->rhs == MFA_RHS_DATABOX) {
      bp.ell(X.Nseg, (int)X.SD, n, p + 1, false);
      bp.ell(X.NsegT, (int)X.SF, (int)X.SD, X.LNsT, false);
      bp.ell(X.Zseg, (int)X.SF, (int)X.SF, X.Fmax, false);
      bp.ell(X.Comb, n, (int)X.SF, 2, false);
      bp.ell(X.Jseg, nif * p, (int)X.SF, 2 * X.Fmax, false);
      bp.ell(X.Omseg, (int)m, (int)X.SF, X.LOm, false);
      X.d_qmap = bp.take<int>(X.SD);
    }
  }
  // global arrays
  const int64_t NC = h->nctrl_total;
  h->c = bp.take<double>(NC);
  h->P = bp.take<double>(NC);
  h->g = bp.take<double>(NC);
  // scratch: the largest intermediate of the N^T Q chain, the decode chain,
  // the sweep chains and the jump chains (simulated with the same rules)
  int64_t s1 = NC, s2 = NC;
  auto upd = [&](int which, int64_t v) {
    if (which == 0) s1 = std::max(s1, v);
    else s2 = std::max(s2, v);
  };
  {
    // both chains run from axis 2 down to the first active axis, whose pass
    // writes the chain's output (c, or the caller's decode buffer) directly
    int first = 0;
    while (first < 2 && !h->ax[first].active) ++first;
    Dims d{{h->ax[0].m, h->ax[1].m, h->ax[2].m}};
    int w = 0;
    for (int ia = 2; ia > first; --ia) {
      if (!h->ax[ia].active) continue;
      d.d[ia] = h->ax[ia].n;
      upd(w, d.total());
      w ^= 1;
    }
    Dims e{{h->ax[0].n, h->ax[1].n, h->ax[2].n}};
    w = 0;
    for (int ia = 2; ia > first; --ia) {
      if (!h->ax[ia].active) continue;
      e.d[ia] = h->ax[ia].m;
      upd(w, e.total());
      w ^= 1;
    }
    for (int a = 0; a < 3; ++a) {
      if (!h->ax[a].active || h->ax[a].B < 2) continue;
      if (h->rhs == MFA_RHS_DATABOX) {
        Dims j{{h->ax[0].SF, h->ax[1].SF, h->ax[2].SF}};
        for (int c = 0; c < 3; ++c)
          if (!h->ax[c].active) j.d[c] = 1;
        j.d[a] = (int64_t)(h->ax[a].B - 1) * p;
        int ww = 0;
        upd(ww, j.total());
        for (int c = 0; c < 3; ++c) {
          if (c == a || !h->ax[c].active) continue;
          ww ^= 1;
          j.d[c] = h->ax[c].m;
          upd(ww, j.total());
        }
      }
      Dims j{{h->ax[0].n, h->ax[1].n, h->ax[2].n}};
      j.d[a] = (int64_t)(h->ax[a].B - 1) * p;
      w = 0;
      upd(w, j.total());
      for (int c = 0; c < 3; ++c) {
        if (c == a || !h->ax[c].active) continue;
        w ^= 1;
        j.d[c] = h->ax[c].m;
        upd(w, j.total());
      }
    }
  }
  if (h->variant == MFA_VARIANT_DECOUPLED) {
    const int64_t cn[3] = {h->ax[0].nv, h->ax[1].nv, h->ax[2].nv};
    chain_scratch(h, cn, &s1, &s2);
  }
  h->s1 = bp.take<double>(s1);
  h->s2 = bp.take<double>(s2);
  h->s1n = s1;
  h->s2n = s2;
  if (h->rhs == MFA_RHS_DATABOX) {
    // every intermediate of a per-subdomain sweep: decode onto the data boxes
    // (n -> SD per axis), N_F^T (SD -> SF), local inverses (SF), combine
    // (SF -> n); both box buffers are sized for the largest one
    int64_t big = 1;
    Dims d{{h->ax[0].n, h->ax[1].n, h->ax[2].n}};
    for (int ia = 2; ia >= 0; --ia) {
      if (!h->ax[ia].active) continue;
      d.d[ia] = h->ax[ia].SD;
      big = std::max(big, d.total());
    }
    for (int ia = 0; ia < 3; ++ia) {
      if (!h->ax[ia].active) continue;
      d.d[ia] = h->ax[ia].SF;
      big = std::max(big, d.total());
    }
    for (int ia = 0; ia < 3; ++ia) {
      if (!h->ax[ia].active) continue;
      d.d[ia] = h->ax[ia].n;
      big = std::max(big, d.total());
    }
    h->b1 = bp.take<double>(big);
    h->b2 = bp.take<double>(big);
    h->b1n = h->b2n = big;
  }
  h->slot_base = bp.take<unsigned long long>(2 * (int64_t)kNumSlots * kSlotCopies);
  h->slots = h->slot_base;
  h->flag = bp.take<int>(4);
  h->hist = bp.take<double>(kHist);
  h->res_slots = bp.take<unsigned long long>(2 * (int64_t)kSlotCopies);
  return bp.off + 256;
}

}  // namespace mfa
