/*
 * mfa.h - C ABI of the MI355X multivariate functional approximation encoder.
 *
 * The library fits a tensor-product B-spline (degree p, clamped uniform knots,
 * all weights W = 1) to data on a regular 1-D, 2-D or 3-D grid with the
 * overlapping additive-Schwarz domain decomposition of Mahadevan, Lenz,
 * Grindeanu and Peterka (arXiv 2210.06528): the control grid is split into
 * axis-aligned subdomains that overlap by `overlap` control points (the
 * shared spans Delta plus the augmented spans delta of Section 2.2); every
 * sweep solves each subdomain's local least-squares problem (eq.
 * minimization-problem) with its neighbours' control points lagged (the
 * block-Jacobi reading of eq. global-system), and the local solutions are
 * combined with the uniform weights 1/n_s of Section 2.3.2 (Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids are C-ordered, last axis contiguous.  Data point i of an axis with
 *    m points sits at parameter u = i/(m-1).  Control point arrays have shape
 *    nctrl[0] x ... x nctrl[dim-1].
 *  - Pointers named *_dev are HIP device pointers on the device that was
 *    current when mfa_create ran; pointers named *_host are host memory.
 *  - All work is ordered on the HIP stream given to mfa_create.  Independent
 *    parts of the setup and of a convergence check run on two auxiliary
 *    streams the library keeps per host thread and device (default priority),
 *    forked from that stream with an event and joined back to it before any
 *    later work on it.  Calls return when the work is enqueued unless stated
 *    otherwise; mfa_create, mfa_encode (to read the convergence metrics) and
 *    mfa_schwarz_step (to fill its statistics) synchronise the stream before
 *    returning.
 *  - The caller owns every buffer passed in, including the workspace; the
 *    library never allocates device memory.  It must outlive the handle.
 *  - Errors: every entry point returns an mfa_status; on failure
 *    mfa_last_error() returns a message for the calling thread.  No C++
 *    exception crosses the ABI.  Calls on one handle must not overlap.
 */
#ifndef MFA_H
#define MFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfa_handle mfa_handle;

typedef enum {
  MFA_OK = 0,
  MFA_EINVAL = -1,    /* invalid argument or problem (message says which)      */
  MFA_ENOMEM = -2,    /* workspace smaller than mfa_workspace_size reported    */
  MFA_EDEVICE = -3,   /* a HIP runtime call failed                             */
  MFA_ENOTCONV = -4,  /* max_sweeps reached with jumps above jump_tol, or NaN  */
  MFA_ESINGULAR = -5  /* a local normal matrix is not positive definite:       */
                      /* some basis function has no data point in its support */
} mfa_status;

typedef enum { MFA_F32 = 0, MFA_F64 = 1 } mfa_dtype;

/* Arithmetic of the sweep.  FP64: everything in float64.  MIXED_*: the
 * residual of the normal equations, the control points and the Cholesky
 * factors stay float64, the Schwarz correction is applied in lower precision
 * and the sweep acts as iterative refinement on the float64 residual.      */
typedef enum {
  MFA_PREC_FP64 = 0,
  MFA_PREC_MIXED_FP32 = 1,
  MFA_PREC_MIXED_BF16 = 2
} mfa_precision;

/* Combine of the local solutions.  AVG: uniform weights 1/n_s over every
 * subdomain whose free set holds the control point (Section 2.3.2).  RAS:
 * restricted, each control point takes its owning subdomain's value.       */
typedef enum { MFA_COMBINE_AVG = 0, MFA_COMBINE_RAS = 1 } mfa_combine;

/* How a sweep forms each subdomain's local right-hand side.
 * NORMAL: from c = N^T Q (computed once per input) minus N^T N P, which
 *         equals the local N_F^T (Q - N P) exactly; Q is read once per encode.
 * DATABOX: decode on every subdomain's data box and form N_F^T (Q - N P)
 *         from the point residual every sweep, as Algorithm 1 is written.  */
typedef enum { MFA_RHS_NORMAL = 0, MFA_RHS_DATABOX = 1 } mfa_rhs;

/* The model the encode builds (Section 2.1; compared in Section 3.1.1).
 * SCHWARZ:   one spline on floating interface knots; the overlapping Schwarz
 *            sweeps of Algorithm 1 make it the single-domain fit (C^{p-1}).
 * DECOUPLED: every subdomain's unconstrained local fit (Algorithm 1's P = 0
 *            branch, floating knots, no exchange), one spline per subdomain;
 *            the decode takes each point from the subdomain that owns it, so
 *            the field is discontinuous at interfaces.  Control points are the
 *            subdomains' free sets side by side along every axis
 *            (sum over blocks of |F_b| per axis).
 * CLAMPED:   every subdomain has its own clamped uniform knots and nctrl[a][b]
 *            control points; neighbours share the control point on their
 *            interface, which takes the input datum there (interfaces sit on
 *            data points, placed in proportion to the blocks' spans); lower-
 *            dimensional interface entities are fitted first and frozen, so
 *            the field is C^0 across interfaces.  sum(nctrl) - (nsub - 1)
 *            control points per axis; `overlap` is not used.
 * The two variants are one-shot fits (no sweeps) in float64: precision must
 * be FP64 and rhs NORMAL; CLAMPED takes no weights.                       */
typedef enum { MFA_VARIANT_SCHWARZ = 0, MFA_VARIANT_DECOUPLED = 1, MFA_VARIANT_CLAMPED = 2 } mfa_variant;

typedef struct {
  int32_t dim;               /* 1, 2 or 3                                           */
  int64_t npts[3];           /* data points per axis (>= nctrl on that axis)        */
  int32_t degree;            /* p >= 1, the same on every axis (Algorithm 1's p)    */
  int32_t nsub[3];           /* subdomains per axis (the paper's N per axis)        */
  const int32_t *nctrl[3];   /* host arrays: owned control points of each
                                subdomain along each axis, length nsub[a]; they
                                sum to the axis' control count (uneven allowed)   */
  int32_t overlap;           /* control points added to each interior side of a
                                subdomain's free set (|Delta| + |delta|);
                                must be >= max(1, floor(p/2)) when nsub[a] > 1     */
  int32_t precision;         /* mfa_precision                                      */
  int32_t combine;           /* mfa_combine                                        */
  int32_t rhs;               /* mfa_rhs                                            */
  double lo[3], hi[3];       /* physical extent of each axis: data point i sits at
                                x = lo + (hi - lo) i/(m-1) (parameter u = i/(m-1)).
                                Only derivative outputs depend on it: they come
                                back with respect to x, d^r/dx^r =
                                (hi - lo)^-r d^r/du^r.  lo == hi (a zeroed struct)
                                means the unit interval: derivatives in u.       */
  const double *weights[3];  /* host arrays or NULL: NURBS weights of each axis'
                                control points (length = the axis' control count,
                                positive and finite).  The basis is then the
                                rational basis of eq. nurbs-basis with the
                                tensor-product weights W = w_0 x w_1 x w_2, i.e.
                                R_a = N_a w_a / sum N_a w_a on every axis; NULL is
                                W = 1 on that axis (plain B-splines).            */
  int32_t variant;           /* mfa_variant value; 0 is the Schwarz encoder        */
} mfa_problem;

#define MFA_MAX_DEGREE 8

typedef struct {
  int32_t sweep;                  /* sweeps done since the last mfa_encode start     */
  int32_t converged;              /* 1 if max_r jump[r] < jump_tol                   */
  double jump[MFA_MAX_DEGREE];    /* normalised interface jumps J_r, r = 0..p-1
                                     (eq. nonlinear-residuals; max over axes and
                                     interfaces of |d^r (L_i - L_j)/du^r| on the
                                     interface, divided by max(S_r, S_0), S_r the
                                     largest r-th derivative control coefficient of
                                     the consensus and S_0 = max |P|)               */
  double max_dP;                  /* max |P_new - P| of the last sweep               */
  double nres_max;                /* max |N^T Q - N^T N P| before the last sweep     */
  double ctrl_max;                /* S_0 = max |P| after the last sweep              */
  double res_max, res_l2;         /* error of the fit after the last sweep against
                                     the data (Algorithm 1's E): max |Q - N P| and
                                     ||Q - N P||_2 over all data points.  Filled by
                                     mfa_schwarz_step; mfa_encode leaves NaN (it
                                     never decodes on the data: mfa_fit_error)     */
} mfa_step_stats;

/* Bytes of device workspace mfa_create needs for this problem.
 * Validates the problem; MFA_EINVAL names the first violated rule:
 * dim not in 1..3, p < 1 or > MFA_MAX_DEGREE, an axis with fewer points than
 * control points, overlap below max(1, floor(p/2)) on a split axis (the
 * floor(p/2) shared spans needed for partition of unity, Section 2.2), an
 * owned block smaller than max(p+1, 2*overlap) on a split axis, a null
 * pointer, a precision/combine/rhs value out of range, an axis extent with
 * hi < lo or a non-finite bound, or a weight that is not positive and
 * finite.                                                                   */
mfa_status mfa_workspace_size(const mfa_problem *prob, size_t *bytes);

/* Control points per axis of the problem's model (dims[a] for a < dim): the
 * axis' control count for SCHWARZ, the free sets side by side for DECOUPLED,
 * sum(nctrl) - (nsub - 1) for CLAMPED.  Host-side planning only.            */
mfa_status mfa_ctrl_dims(const mfa_problem *prob, int64_t dims[3]);

/* Plan the subdomains (Section 2.2), evaluate the Cox-de Boor basis at every
 * data point (Section 2.1), assemble the banded per-axis normal matrices
 * N_a^T N_a with wavefront reductions, factor every subdomain's local normal
 * matrix with a batched banded Cholesky (Section 2.3.1) and build the
 * per-axis Schwarz operators; everything is ordered on `hip_stream` (a
 * hipStream_t, or NULL for the default stream; the three axes' setup runs
 * concurrently on it and two auxiliary streams).  `workspace` is a device buffer of at
 * least mfa_workspace_size bytes, 256-byte aligned.  Synchronises the stream.
 * Returns MFA_ESINGULAR when a local normal matrix is not positive definite.
 * On success *out owns no memory but the small host-side handle.           */
mfa_status mfa_create(const mfa_problem *prob, void *workspace, size_t bytes,
                      void *hip_stream, mfa_handle **out);

/* mfa_create without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture around the call, serving loops and
 * harnesses that forbid hipMalloc).  The handle's workspace is the library's
 * own file-scope device array of MFA_NOALLOC_MAX_BYTES bytes (256 MiB, one
 * copy per device, held from the first use of the library on that device
 * until the process ends); problems whose mfa_workspace_size exceeds it are
 * rejected with MFA_ENOMEM before any device work.  Otherwise as mfa_create
 * (same plan, setup kernels and results), except that every launch stays on
 * `hip_stream`: no auxiliary streams are forked, the residual stencil takes
 * its untimed default chunking, and the call creates no HIP streams or events
 * and calls no allocating routine (hipMalloc, hipFree, torch).  The array
 * keeps the previous contents; everything that must start at zero is cleared
 * on the stream by the setup.
 * Sharing: all no-allocation handles on a device share that one array.
 * Creating one claims the array: calls on an older no-allocation handle of
 * the same device then fail with MFA_EINVAL (mfa_destroy still releases it),
 * and calls that overlap on the array (two streams, two threads) race.      */
#define MFA_NOALLOC_MAX_BYTES (256u * 1024u * 1024u)
mfa_status mfa_create_noalloc(const mfa_problem *prob, void *hip_stream, mfa_handle **out);

/* Algorithm 1 on the data q_dev (npts[0] x ... float32 or float64 device
 * array): start from the control points set by mfa_set_ctrl, else from zero
 * (the first sweep is then the decoupled local fit), and sweep until
 * max_r J_r < jump_tol or max_sweeps.  The jumps are evaluated every
 * `check_every` sweeps.  check_every <= 0 predicts the checks: the first at
 * sweep 6; after a check at sweep k with largest jump J the next comes
 * ceil(log(jump_tol / J) / log(rho)) sweeps later (clamped to 1..32), rho =
 * sqrt(max|dP_k| / max|dP_{k-2}|) the decay of the corrections every sweep
 * records (4 sweeps later when no decay is seen).  The count predicted at
 * the first check is rounded down instead when an axis has four or more
 * subdomains (the decay is still speeding up there at sweep 6).  The stop
 * may come a few sweeps after the first sweep that met the tolerance.  jump_tol <= 0 runs exactly max_sweeps sweeps.  `last` (may be
 * NULL) receives the statistics of the last checked sweep.  Returns
 * MFA_ENOTCONV if the tolerance was not met (the control points are still
 * the last iterate) or a non-finite value appeared.                         */
mfa_status mfa_encode(mfa_handle *h, const void *q_dev, mfa_dtype q_dtype,
                      int32_t max_sweeps, double jump_tol, int32_t check_every,
                      mfa_step_stats *last);

/* One sweep of Algorithm 1 from the current control points.  q_dev as in
 * mfa_encode; q_dev == NULL reuses the data of the previous call on this
 * handle.  Fills *out (may be NULL) including the jumps.  Synchronises.     */
mfa_status mfa_schwarz_step(mfa_handle *h, const void *q_dev, mfa_dtype q_dtype,
                            mfa_step_stats *out);

/* Algorithm 1's error vector E = Q - N P of the current control points
 * against the data of the last mfa_encode / mfa_schwarz_step on this handle
 * (that buffer must still hold the data): *res_max = max |E| and *res_l2 =
 * ||E||_2 over every data point.  One decode of the spline on the data grid,
 * compared with Q and reduced on the device (nothing is stored; costs about
 * one mfa_decode).  Synchronises the stream.  EINVAL when no data was loaded.
 * mfa_schwarz_step runs the same pass for its statistics.                   */
mfa_status mfa_fit_error(mfa_handle *h, double *res_max, double *res_l2);

/* Evaluate the consensus spline (or, with deriv != NULL, the mixed partial
 * derivative of orders deriv[0..dim-1] with respect to the parameters u_a,
 * each <= p) at every grid point into out_dev (npts[0] x ... of out_dtype).
 * This is the decode of Section 2.1 (eq. nurbs-basis).                      */
mfa_status mfa_decode(mfa_handle *h, void *out_dev, mfa_dtype out_dtype,
                      const int32_t *deriv);

/* Decode at arbitrary parameter points (Section 2.1: the tensor-product
 * B-spline of eq. nurbs-basis with W = 1, evaluated away from the grid, the
 * analysis use of the fitted model).  For point i with parameters
 * u_dev[i*dim + a] (row-major, npoints x dim, device memory, float64):
 *   out[i] = sum_k P[k] prod_a d^{r_a}/du_a^{r_a} N_{k_a,p}(u_a)
 * with r_a = deriv[a] (0..p; nullable = values), spans taken right-continuous
 * as for the data grid (u = t_j belongs to span j, u = 1 to span n-1).
 * Parameters outside [0, 1] are clamped to the nearest end.  out_dev holds
 * npoints values of out_dtype.  Asynchronous on the handle's stream; reads
 * the current control points.  EINVAL for null pointers, npoints < 0 or a
 * derivative order outside 0..p.  */
mfa_status mfa_decode_points(mfa_handle *h, const double *u_dev, int64_t npoints, void *out_dev,
                             mfa_dtype out_dtype, const int32_t *deriv);

/* Copy the control points (float64, nctrl[0] x ...) out of / into the handle
 * ("write MFA to disk" of Algorithm 1; set_ctrl is a warm start or refit).
 * on_device != 0: the pointer is a device pointer; otherwise host memory
 * (the copy then completes before the call returns).  mfa_set_ctrl with
 * ctrl == NULL copies nothing and makes the next mfa_encode start from the
 * control points the handle already holds (Algorithm 1's branch for P != 0:
 * a refit of new data on a resident model, without the decoupled first
 * sweep).                                                                   */
mfa_status mfa_get_ctrl(mfa_handle *h, double *ctrl, int32_t on_device);
mfa_status mfa_set_ctrl(mfa_handle *h, const double *ctrl, int32_t on_device);

/* Move the handle's work to another HIP stream of the same device (a
 * resident model driven from another thread or slot).  Synchronises the old
 * stream first, so no work is left on it; later calls enqueue on
 * `hip_stream`.                                                             */
mfa_status mfa_set_stream(mfa_handle *h, void *hip_stream);

/* Copy an intermediate table into host memory for inspection (tests):
 *  MFA_T_BASIS   basis values, axis `axis`: npts x (p+1), row i holds
 *                N_{s-p..s}(u_i) with s the span of u_i (Section 2.1)
 *  MFA_T_SPAN    spans as float64, npts values
 *  MFA_T_GRAM    lower band of N_a^T N_a: (p+1) x nctrl, band[t][k] = A[k+t][k]
 *  MFA_T_CHOL    banded Cholesky factor of subdomain `block` on axis `axis`,
 *                lower band (p+1) x |F|
 *  MFA_T_INV     inverse of that local normal matrix, |F| x |F| row-major
 *  MFA_T_RHS     N^T Q of the last input, float64 control array
 * `count` is the capacity of host_out in doubles; the needed count is
 * written to *needed (may be NULL).  Synchronises the stream.              */
typedef enum {
  MFA_T_BASIS = 0, MFA_T_SPAN = 1, MFA_T_GRAM = 2, MFA_T_CHOL = 3,
  MFA_T_INV = 4, MFA_T_RHS = 5
} mfa_table;
mfa_status mfa_inspect(mfa_handle *h, int32_t table, int32_t axis, int32_t block,
                       double *host_out, size_t count, size_t *needed);

/* Per-kernel event timing (measurement support).  class_mask selects the
 * kernel classes below (bit c for class c; MFA_K_ALL for every class, 0 to
 * disable): the library records a HIP event pair on its stream around every
 * launch of a selected class; mfa_kernel_time synchronises the stream and
 * returns the summed duration in milliseconds and the number of launches of
 * one class since timing was set (or since the class was last read, which
 * resets it).  Disabled by default; every timed launch costs two event
 * records on the stream.  */
typedef enum {
  MFA_K_PROJECT = 0,   /* c = N^T Q passes                                 */
  MFA_K_RESID = 1,     /* residual stencil g = c - N^T N P                 */
  MFA_K_CORRECT = 2,   /* Schwarz correction passes (banded solves)        */
  MFA_K_METRICS = 3,   /* interface jumps and derivative scales            */
  MFA_K_DECODE = 4,    /* decode passes                                    */
  MFA_K_COUNT = 5,
  MFA_K_ALL = (1 << 5) - 1
} mfa_kernel_class;
mfa_status mfa_set_timing(mfa_handle *h, int32_t class_mask);
mfa_status mfa_kernel_time(mfa_handle *h, int32_t kclass, double *total_ms, int64_t *launches);

/* Sampled timing: counting the launches of each timed class from 0 (from
 * this call or the last mfa_set_timing), only launches first, first + every,
 * first + 2 every, ... get the event pair (every = 1, first = 0, the
 * default, times them all); the launch count mfa_kernel_time returns is the
 * number timed.  Each event record costs the stream a few microseconds, so a
 * caller that times a kernel launched many times over can sample it; varying
 * `first` over repeated runs samples every launch position equally.  Needs
 * every >= 1 and 0 <= first < every, else MFA_EINVAL.  */
mfa_status mfa_set_timing_every(mfa_handle *h, int32_t every, int32_t first);

/* Release the handle (not the caller-owned workspace).  NULL is ignored.   */
void mfa_destroy(mfa_handle *h);

/* Message describing the last failure on the calling thread ("" if none).  */
const char *mfa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFA_H */
