// Internal declarations of the MFA library (host planner, device tables,
// kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mfa.h"

namespace mfa {

constexpr int kMaxP = MFA_MAX_DEGREE;

// Row-sparse operator along one axis in ELL layout: row r has len[r] <= L
// nonzeros at columns col[r*L + t] with values val[r*L + t].
struct Ell {
  int R = 0;        // rows (output length along the axis)
  int C = 0;        // columns (input length along the axis)
  int L = 0;        // max nonzeros per row
  int *len = nullptr;
  int *col = nullptr;
  double *val = nullptr;
  float *valf = nullptr;   // float copy (mixed precision), may be null
};

// Index ranges of one subdomain along one axis (Section 2.2).
struct Block {
  int c0, c1;          // owned control points [c0, c1)
  int F0, F1;          // free set: owned plus `overlap` on interior sides
  int E0, E1;          // free set plus the p ghost control points per side
  int64_t D0, D1;      // data points in the support of the free set
  int64_t own0, own1;  // owned data points (a partition of the axis)
};

// Plan and device tables of one axis.  Axes are stored innermost-last as
// internal axes 0..2; a problem of dimension d uses internal axes 3-d..2 and
// the others have length 1 and no operators.
struct Axis {
  bool active = false;
  int64_t m = 1;        // data points
  int n = 1;            // control points
  int B = 1;            // subdomains
  double dscale = 1.0;  // du/dx = 1 / (hi - lo): derivative tables carry dscale^r
  std::vector<double> w;          // NURBS weights (empty: all 1)
  double *d_w = nullptr;          // device copy of w (null when unweighted)
  // variants (DECOUPLED, CLAMPED): the model's control count along the axis
  // and its fit / decode / interface-jump operators
  int nv = 0;
  std::vector<int> ccut;          // CLAMPED: data index of each block boundary (B+1)
  std::vector<int> coff, csz;     // CLAMPED: first control point and size of each block
  int *d_ccut = nullptr, *d_coff = nullptr, *d_csz = nullptr;
  int64_t LLv = 0;                // widest fit row (data points of one block)
  Ell Lv;                         // nv x m: data -> control points
  Ell Nv[kMaxP + 1];              // m x nv: decode, derivative order 0..p
  Ell Jv;                         // (B-1)p x nv: interface derivative differences
  std::vector<Block> blk;
  std::vector<int> ns;            // subdomains whose free set holds each ctrl
  std::vector<int> blo, bhi;      // first / last block whose free set holds ctrl k
  std::vector<int> owner;         // block owning ctrl k
  std::vector<int> pown;          // block owning data point i
  std::vector<double> ustar;      // interface parameters (B-1)
  std::vector<int> span_if;       // span of each interface parameter
  int64_t LNT = 0, LM = 0, LOm = 0, LJ = 0;
  int64_t Fmax = 0;
  std::vector<int64_t> chol_off, inv_off;   // per-block offsets (doubles)
  int64_t chol_total = 0, inv_total = 0;
  int64_t ND = 0;                            // rows of the derivative-coefficient table
  // DATABOX segmented layouts
  int64_t SD = 0, SF = 0;                    // sum of |D_b| and of |F_b|
  std::vector<int64_t> doff, foff;           // segment offsets per block
  int64_t LNsT = 0;

  // device pointers (inside the workspace)
  int *d_span = nullptr;
  double *d_bas = nullptr;           // m x (p+1), values
  double *d_gram = nullptr;          // (p+1) x n lower band
  double *d_chol = nullptr;
  double *d_inv = nullptr;
  int *d_blk = nullptr;              // per block: c0 c1 F0 F1 own0 own1 D0 D1 (int)
  int *d_blo = nullptr, *d_bhi = nullptr, *d_owner = nullptr, *d_pown = nullptr;
  int *d_ns = nullptr;
  double *d_ustar = nullptr;
  int *d_span_if = nullptr;
  double *d_dbas_if = nullptr;       // (B-1) x p x (p+1)
  int *d_gidJ = nullptr;             // J row -> r
  int *d_gidD = nullptr;             // D row -> r
  double *d_acoef = nullptr;         // (2p+1) x n stencil rows of A (identity if inactive)
  int *d_choff = nullptr;            // per-block offset of the Cholesky factor
  int *d_foff = nullptr;             // per-block offset into d_rdiag (sum of earlier |F_b|)
  double *d_rdiag = nullptr;         // 1 / L_jj of every block's factor
  double *d_omT = nullptr;           // Om values transposed (L x m)
  // mixed BF16: dense split-BF16 copy of M (hi then lo; rows padded to 16,
  // npad columns) and the K range of every 16-row tile
  int npad = 0;
  void *d_Mb = nullptr;
  int *d_klo = nullptr, *d_knc = nullptr;
  Ell N[kMaxP + 1];                  // decode tables, derivative order 0..p
  Ell NT, A, M, Om, J, D;
  // DATABOX tables
  Ell Nseg, NsegT, Zseg, Comb, Jseg, Omseg;
  int *d_qmap = nullptr;             // segmented data row -> data point index
};

struct Handle {
  mfa_problem prob{};
  int dim = 0, p = 0, overlap = 0, precision = 0, combine = 0, rhs = 0, variant = 0;
  Axis ax[3];
  hipStream_t stream = nullptr;
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int64_t nctrl_total = 1, npts_total = 1;
  // state
  double *c = nullptr;      // N^T Q
  double *P = nullptr;      // consensus control points
  double *g = nullptr;      // N^T Q - N^T N P
  double *s1 = nullptr, *s2 = nullptr;   // scratch
  int64_t s1n = 0, s2n = 0;
  // DATABOX scratch
  double *b1 = nullptr, *b2 = nullptr;
  int64_t b1n = 0, b2n = 0;
  // reductions, see kSlot*: two sets of kNumSlots * kSlotCopies, used by
  // alternate sweeps (slots points to the current sweep's set)
  unsigned long long *slot_base = nullptr;
  unsigned long long *slots = nullptr;
  int *flag = nullptr;                   // setup error flag
  double *hist = nullptr;                // max |correction| of recent sweeps (ring of kHist)
  unsigned long long *res_slots = nullptr;   // data-residual reduction (2 x kSlotCopies)
  size_t upload_bytes = 0;               // host-planned tables: workspace bytes [0, upload_bytes)
  bool fuse21 = true;                    // fused axis-2/axis-1 correction when it applies
  bool have_rhs = false;
  const void *q = nullptr;  // data of the last encode / step (read every sweep in DATABOX mode)
  int q_dtype = 0;
  int g_type = 0;           // element type of g: 0 float64, 1 float32, 2 bfloat16
  bool warm = false;        // P was set by mfa_set_ctrl: the next encode starts there
  bool p_zero = false;      // P still holds the zeros mfa_create wrote (nothing has written it since)
  bool p_known_zero = false;  // P = 0 for the next sweep (cold start of an encode)
  bool serial = false;      // every launch on `stream` (no auxiliary streams or tuner events)
  uint64_t noalloc_gen = 0; // nonzero: the workspace is the device's no-allocation array,
                            // claimed by this handle as generation noalloc_gen
  int sweep = 0;
  // per-class event timing
  int timing = 0;                        // mask of timed kernel classes
  int timing_every = 1;                  // time one launch in this many per class,
  int timing_first = 0;                  // starting with this one (< timing_every)
  int64_t timing_seen[MFA_K_COUNT] = {}; // launches per class since timing was set
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[MFA_K_COUNT];
  std::vector<hipEvent_t> ev_pool;
  ~Handle();
};

// Records an event pair around the launches in its scope when timing is on.
struct TimeScope {
  Handle &h;
  int cls;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimeScope(Handle &hh, int c);
  ~TimeScope();
};

// reduction slots (double bit patterns of non-negative maxima)
constexpr int kSlotMaxDP = 0;
constexpr int kSlotNres = 1;
constexpr int kSlotCtrl = 2;
constexpr int kSlotJ = 8;                       // + a*kMaxP + r
constexpr int kSlotS = kSlotJ + 3 * kMaxP;      // + a*kMaxP + r
constexpr int kNumSlots = kSlotS + 3 * kMaxP;
// each logical slot has kSlotCopies physical copies (atomics spread over them
// to avoid serialising on one address); readers take the max over copies
constexpr int kSlotCopies = 64;

// ---------------------------------------------------------------- planner
// Fills h->ax[*] host-side plan; returns an error message or "".
std::string plan_problem(const mfa_problem &prob, Handle *h);
// Lays out the workspace; with base == nullptr only counts bytes.
size_t layout_workspace(Handle *h, char *base);

// The device's no-allocation array (MFA_NOALLOC_MAX_BYTES, 256-byte
// aligned) for the current device: its device address and a new generation
// number that marks the array as claimed by the caller; noalloc_current
// returns the last generation handed out on `device` (0 if none).
hipError_t noalloc_scratch(void **ptr, uint64_t *gen);
uint64_t noalloc_current(int device);

// ---------------------------------------------------------------- kernels
// EPI_RESID32 / EPI_RESID64: `sub` is the data Q (float32 / float64); the
// pass stores nothing and reduces max |Q - value| and sum (Q - value)^2 into
// slots[0..kSlotCopies) and slots[kSlotCopies..2 kSlotCopies)
enum Epi { EPI_STORE = 0, EPI_SUBFROM = 1, EPI_ADDTO = 2, EPI_MAXABS = 3, EPI_STOREMAX = 4,
           EPI_RESID32 = 5, EPI_RESID64 = 6 };

struct Dims {
  int64_t d[3];
  int64_t total() const { return d[0] * d[1] * d[2]; }
};

// out = op applied along internal axis `ax` of `in` (dims `in_dims`), with
// the chosen epilogue.  Tin/Tout in {float, double}.
template <typename Tin, typename Tout>
hipError_t launch_pass(hipStream_t st, const Tin *in, Dims in_dims, int ax, const Ell &op,
                       Tout *out, int epi, const double *sub, unsigned long long *slots,
                       int slot_base, const int *gid, int gaxis);

hipError_t launch_fill(hipStream_t st, double *x, int64_t n, double v);
// r = Q[qmap0[x0], qmap1[x1], qmap2[x2]] - r on a segmented data-box array
template <typename TQ>
hipError_t launch_box_resid(hipStream_t st, const TQ *q, Dims qd, double *r, Dims rd,
                            const int *qm0, const int *qm1, const int *qm2);
// zero n reduction slots; first record the max |correction| held in the set
// `from` (slot kSlotMaxDP, the previous sweep's) into hist[idx] when hist is
// given
constexpr int kHist = 64;
hipError_t launch_zero_slots(hipStream_t st, unsigned long long *slots, int n, double *hist = nullptr,
                             int idx = 0, const unsigned long long *from = nullptr);
// Slot bookkeeping a sweep's residual kernel does in its first workgroup:
// record the previous sweep's max |correction| (set `prev`) into hist[idx]
// (hist may be null), then clear `prev`, the set the next sweep uses.
struct SlotTurn {
  unsigned long long *prev = nullptr;
  double *hist = nullptr;
  int idx = 0;
};
hipError_t launch_maxabs(hipStream_t st, const double *x, int64_t n, unsigned long long *slot);
// the maxima of nslots slots (ncopies copies each) and one extra value into
// out[0..nslots] (pinned host memory): one small launch instead of a copy of
// every slot copy to pageable memory
hipError_t launch_pack_slots(hipStream_t st, const unsigned long long *slots, int nslots, int ncopies,
                             const double *extra, double *out);
constexpr int kPinnedDoubles = 512;   // per thread and device (pinned_block)
// kPinnedDoubles doubles of pinned host memory for this host thread and
// device, allocated on first use and kept for the life of the process
// (nullptr if the allocation fails; callers then copy to pageable memory)
double *pinned_block(int device);

// setup kernels (one axis at a time)
// one copy of every host-planned table (block bounds, owners, n_s, interface
// parameters, identity stencil rows of inactive axes) into the workspace
// Copy the plan tables into the workspace (asynchronous on h->stream): `img`
// holds the host image and must live until the stream has been synchronised.
hipError_t upload_plan(Handle *h, std::vector<char> &img);
// decode at arbitrary parameter points (npts x dim, float64, device)
hipError_t launch_decode_points(Handle &h, const double *u, int64_t npts, void *out, bool f32,
                                const int r[3]);
hipError_t setup_axes(Handle *h, hipStream_t st);   // every active axis, one launch per stage
// operator tables of the DECOUPLED / CLAMPED variants (after setup_axis for
// DECOUPLED; alone for CLAMPED)
hipError_t setup_variant_axis(Handle *h, int a, hipStream_t st);

// sweep kernels
template <typename TG>
hipError_t launch_resid(hipStream_t st, int p, const double *Pc, const double *c, TG *g,
                        const double *A0, const double *A1, const double *A2, int n0, int n1, int n2,
                        unsigned long long *slots, const SlotTurn &turn = SlotTurn{},
                        bool may_tune = true);
// the residual at P = 0: g = c and max |g| into slot kSlotNres of `slots`
template <typename TG>
hipError_t launch_resid_zero(hipStream_t st, const double *c, TG *g, int64_t n, unsigned long long *slots);
template <typename TI, typename TO, typename TC>
hipError_t launch_bsolve(hipStream_t st, const TI *in, TO *out, double *pc, int axis, int n0, int n1,
                         int n2, int p, const Axis &X, int combine, unsigned long long *slots);
// convergence metrics
hipError_t launch_deriv_scale(Handle &h);
hipError_t launch_jump_expand(Handle &h, int a, const double *U);
template <typename TG>
hipError_t launch_jump_project(Handle &h, int a, const TG *g, double *U);

// mixed BF16 correction on the matrix cores
size_t mfma_lds(int npad);
// streaming projection / decode between the data grid and the control grid
// (axes 1 and 2 active, p <= 6); hipErrorNotSupported when a shape needs the
// generic pass chain instead (nothing is launched then)
bool grid_pass_ok(const Handle &h);
hipError_t launch_project_grid(Handle &h, const void *q, bool f32);
// rs != nullptr: `out` is the data Q (float32 when f32) and the decoded values
// are only compared with it: max |Q - N P| and sum (Q - N P)^2 go to rs
// (kSlotCopies copies each, max then sum)
hipError_t launch_decode_grid(Handle &h, void *out, bool f32, const int r[3],
                              unsigned long long *rs = nullptr);
bool mfma_fits(int npad);
hipError_t setup_mfma_axes(Handle *h, hipStream_t st);
// axes 2 and 1 of the split-BF16 correction in one pass (3-D problems)
// (and, in *maxnc when given, the most 32-column K chunks of one M_2 tile)
int fuse21_ldw(const Handle &h, int *maxnc = nullptr);
bool mfma_fused21_ok(const Handle &h);
hipError_t launch_mfma_fused21(Handle &h, const float *in, float *out);
hipError_t launch_mfma_correct(Handle &h, int axis, const float *in, float *out, bool add);

// LDS bytes the banded-solve kernel needs for segments of length fmax
bool bsolve_seg_ok(const Axis &X);
inline size_t bsolve_lds(int64_t fmax, int p, size_t elem) {
  return (size_t)2 * fmax * 65 * elem + sizeof(double) * (size_t)(p + 2) * fmax;
}

}  // namespace mfa
