"""ctypes binding of libmfa.so (the C ABI declared in include/mfa.h).

Argument marshalling only: every step of the encoder runs in the HIP library.
PyTorch supplies device memory (the workspace, inputs, outputs) and the HIP
stream.  Loading fails loudly when the library has not been built; there is
no fallback.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfa.so")

MFA_OK, MFA_EINVAL, MFA_ENOMEM, MFA_EDEVICE, MFA_ENOTCONV, MFA_ESINGULAR = 0, -1, -2, -3, -4, -5
MFA_F32, MFA_F64 = 0, 1
PRECISION = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2}
COMBINE = {"avg": 0, "ras": 1}
RHS = {"normal": 0, "databox": 1}
VARIANT = {"schwarz": 0, "decoupled": 1, "clamped": 2}
TABLES = {"basis": 0, "span": 1, "gram": 2, "chol": 3, "inv": 4, "rhs": 5}
MAX_DEGREE = 8

STATUS_NAMES = {0: "MFA_OK", -1: "MFA_EINVAL", -2: "MFA_ENOMEM", -3: "MFA_EDEVICE",
                -4: "MFA_ENOTCONV", -5: "MFA_ESINGULAR"}

# every entry point the header declares
EXPORTS = ["mfa_workspace_size", "mfa_create", "mfa_encode", "mfa_schwarz_step", "mfa_decode",
           "mfa_get_ctrl", "mfa_set_ctrl", "mfa_inspect", "mfa_set_timing", "mfa_set_timing_every",
           "mfa_kernel_time", "mfa_decode_points", "mfa_create_noalloc", "mfa_fit_error", "mfa_set_stream",
           "mfa_ctrl_dims",
           "mfa_destroy", "mfa_last_error"]
NOALLOC_MAX_BYTES = 256 * 1024 * 1024   # MFA_NOALLOC_MAX_BYTES
KERNEL_CLASSES = {"project": 0, "resid": 1, "correct": 2, "metrics": 3, "decode": 4}


class mfa_problem(ctypes.Structure):
    _fields_ = [
        ("dim", c_int32),
        ("npts", c_int64 * 3),
        ("degree", c_int32),
        ("nsub", c_int32 * 3),
        ("nctrl", POINTER(c_int32) * 3),
        ("overlap", c_int32),
        ("precision", c_int32),
        ("combine", c_int32),
        ("rhs", c_int32),
        ("lo", c_double * 3),
        ("hi", c_double * 3),
        ("weights", POINTER(c_double) * 3),
        ("variant", c_int32),
    ]


class mfa_step_stats(ctypes.Structure):
    _fields_ = [
        ("sweep", c_int32),
        ("converged", c_int32),
        ("jump", c_double * MAX_DEGREE),
        ("max_dP", c_double),
        ("nres_max", c_double),
        ("ctrl_max", c_double),
        ("res_max", c_double),
        ("res_l2", c_double),
    ]

    def as_dict(self, p):
        return {"sweep": self.sweep, "converged": bool(self.converged),
                "jump": [self.jump[r] for r in range(p)], "max_dP": self.max_dP,
                "nres_max": self.nres_max, "ctrl_max": self.ctrl_max,
                "res_max": self.res_max, "res_l2": self.res_l2}


class MfaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libmfa.so once; raise if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run paper_2210_06528_amd.build.build()")
    # torch brings its own HIP runtime (same soname); load it first so that the
    # library binds to that one instance instead of a second copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    lib.mfa_workspace_size.argtypes = [POINTER(mfa_problem), POINTER(c_size_t)]
    lib.mfa_workspace_size.restype = c_int32
    lib.mfa_ctrl_dims.argtypes = [POINTER(mfa_problem), POINTER(c_int64)]
    lib.mfa_ctrl_dims.restype = c_int32
    lib.mfa_create.argtypes = [POINTER(mfa_problem), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.mfa_create.restype = c_int32
    lib.mfa_create_noalloc.argtypes = [POINTER(mfa_problem), c_void_p, POINTER(c_void_p)]
    lib.mfa_create_noalloc.restype = c_int32
    lib.mfa_encode.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_double, c_int32,
                               POINTER(mfa_step_stats)]
    lib.mfa_encode.restype = c_int32
    lib.mfa_schwarz_step.argtypes = [c_void_p, c_void_p, c_int32, POINTER(mfa_step_stats)]
    lib.mfa_schwarz_step.restype = c_int32
    lib.mfa_fit_error.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double)]
    lib.mfa_fit_error.restype = c_int32
    lib.mfa_decode.argtypes = [c_void_p, c_void_p, c_int32, POINTER(c_int32)]
    lib.mfa_decode.restype = c_int32
    lib.mfa_decode_points.argtypes = [c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_int32,
                                      POINTER(c_int32)]
    lib.mfa_decode_points.restype = c_int32
    lib.mfa_get_ctrl.argtypes = [c_void_p, c_void_p, c_int32]
    lib.mfa_get_ctrl.restype = c_int32
    lib.mfa_set_ctrl.argtypes = [c_void_p, c_void_p, c_int32]
    lib.mfa_set_ctrl.restype = c_int32
    lib.mfa_set_stream.argtypes = [c_void_p, c_void_p]
    lib.mfa_set_stream.restype = c_int32
    lib.mfa_inspect.argtypes = [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double), c_size_t,
                                POINTER(c_size_t)]
    lib.mfa_inspect.restype = c_int32
    lib.mfa_set_timing.argtypes = [c_void_p, c_int32]
    lib.mfa_set_timing.restype = c_int32
    lib.mfa_set_timing_every.argtypes = [c_void_p, c_int32, c_int32]
    lib.mfa_set_timing_every.restype = c_int32
    lib.mfa_kernel_time.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]
    lib.mfa_kernel_time.restype = c_int32
    lib.mfa_destroy.argtypes = [c_void_p]
    lib.mfa_destroy.restype = None
    lib.mfa_last_error.argtypes = []
    lib.mfa_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status):
    if status != MFA_OK:
        raise MfaError(status, load().mfa_last_error().decode())
    return status


def make_problem(npts, degree, sizes, overlap, precision="fp64", combine="avg", rhs="normal",
                 extent=None, weights=None, variant="schwarz"):
    """Build an mfa_problem; the returned tuple keeps the size arrays alive.
    extent: optional per-axis (lo, hi) physical bounds (derivatives in x).
    weights: optional per-axis NURBS weights (None or a sequence of n_a)."""
    dim = len(npts)
    prob = mfa_problem()
    prob.dim = dim
    keep = []
    for a in range(3):
        prob.npts[a] = int(npts[a]) if a < dim else 1
        if a < dim:
            arr = (c_int32 * len(sizes[a]))(*[int(s) for s in sizes[a]])
            keep.append(arr)
            prob.nsub[a] = len(sizes[a])
            prob.nctrl[a] = ctypes.cast(arr, POINTER(c_int32))
        else:
            prob.nsub[a] = 1
            prob.nctrl[a] = None
    prob.degree = int(degree)
    prob.overlap = int(overlap)
    prob.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    prob.combine = COMBINE[combine] if isinstance(combine, str) else int(combine)
    prob.rhs = RHS[rhs] if isinstance(rhs, str) else int(rhs)
    if extent is not None:
        for a, (lo, hi) in enumerate(extent):
            prob.lo[a], prob.hi[a] = float(lo), float(hi)
    prob.variant = VARIANT[variant] if isinstance(variant, str) else int(variant)
    for a in range(3):
        prob.weights[a] = None
    if weights is not None:
        for a, wa in enumerate(weights):
            if wa is None:
                continue
            arr = (c_double * len(wa))(*[float(v) for v in wa])
            keep.append(arr)
            prob.weights[a] = ctypes.cast(arr, POINTER(c_double))
    return prob, keep


def workspace_size(npts, degree, sizes, overlap, precision="fp64", combine="avg", rhs="normal",
                   variant="schwarz"):
    """Bytes of workspace (host-side planning only; raises MfaError on bad input)."""
    prob, keep = make_problem(npts, degree, sizes, overlap, precision, combine, rhs,
                              variant=variant)
    out = c_size_t(0)
    check(load().mfa_workspace_size(ctypes.byref(prob), ctypes.byref(out)))
    return out.value


def ctrl_dims_of(prob):
    """Control points per axis of a problem's model (mfa_ctrl_dims)."""
    dims = (c_int64 * 3)()
    check(load().mfa_ctrl_dims(ctypes.byref(prob), dims))
    return tuple(int(dims[a]) for a in range(prob.dim))


class Encoder:
    """One MFA problem on one GPU: owns the handle and its torch workspace.

    noalloc=True creates the handle with mfa_create_noalloc: no workspace is
    allocated; the handle uses the library's per-device array."""

    def __init__(self, npts, degree, sizes, overlap, precision="fp64", combine="avg",
                 rhs="normal", device="cuda:0", stream=None, noalloc=False, extent=None,
                 weights=None, variant="schwarz"):
        import torch
        self.torch = torch
        self.lib = load()
        self.npts = tuple(int(m) for m in npts)
        self.dim = len(self.npts)
        self.degree = int(degree)
        self.sizes = [list(map(int, s)) for s in sizes]
        self.nctrl = tuple(sum(s) for s in self.sizes)
        self.device = torch.device(device)
        self.prob, self._keep = make_problem(npts, degree, sizes, overlap, precision, combine, rhs,
                                             extent, weights, variant)
        self.nctrl = ctrl_dims_of(self.prob)
        nbytes = c_size_t(0)
        check(self.lib.mfa_workspace_size(ctypes.byref(self.prob), ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self.noalloc = bool(noalloc)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if self.noalloc:
                self.workspace = None
                h = c_void_p(0)
                check(self.lib.mfa_create_noalloc(ctypes.byref(self.prob),
                                                  c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
                self.handle = h
                return
            self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            h = c_void_p(0)
            check(self.lib.mfa_create(ctypes.byref(self.prob), c_void_p(self._ws_ptr),
                                      c_size_t(self.ws_bytes), c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)))
        self.handle = h

    def recreate(self):
        """Destroy and re-create the handle on the same workspace (setup again)."""
        self.close()
        h = c_void_p(0)
        if self.noalloc:
            with self.torch.cuda.device(self.device):
                check(self.lib.mfa_create_noalloc(ctypes.byref(self.prob),
                                                  c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
            self.handle = h
            return
        check(self.lib.mfa_create(ctypes.byref(self.prob), c_void_p(self._ws_ptr),
                                  c_size_t(self.ws_bytes), c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(h)))
        self.handle = h

    # -- helpers
    def _dt(self, t):
        torch = self.torch
        if t.dtype == torch.float32:
            return MFA_F32
        if t.dtype == torch.float64:
            return MFA_F64
        raise TypeError("data must be float32 or float64")

    def _check_q(self, q):
        if tuple(q.shape) != self.npts or not q.is_contiguous() or q.device != self.device:
            raise ValueError(f"data must be a contiguous {self.npts} tensor on {self.device}")

    def _check_out(self, out, shape):
        """An output tensor must be float32/float64, contiguous, of `shape`,
        on this encoder's device; returns its mfa_dtype."""
        if not isinstance(out, self.torch.Tensor) or out.device != self.device:
            raise ValueError(f"output must be a tensor on {self.device}")
        if tuple(out.shape) != tuple(shape) or not out.is_contiguous():
            raise ValueError(f"output must be a contiguous tensor of shape {tuple(shape)}")
        return self._dt(out)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.mfa_destroy(self.handle)
            self.handle = c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the ABI
    def encode(self, q, max_sweeps, jump_tol=0.0, check_every=1, raise_on_notconv=True):
        self._check_q(q)
        self._q = q   # the handle reads the data again (steps without q, fit_error)
        st = mfa_step_stats()
        s = self.lib.mfa_encode(self.handle, c_void_p(q.data_ptr()), self._dt(q), int(max_sweeps),
                                float(jump_tol), int(check_every), ctypes.byref(st))
        if s == MFA_ENOTCONV and not raise_on_notconv:
            return st.as_dict(self.degree)
        check(s)
        return st.as_dict(self.degree)

    def step(self, q=None):
        st = mfa_step_stats()
        if q is not None:
            self._check_q(q)
            self._q = q
            check(self.lib.mfa_schwarz_step(self.handle, c_void_p(q.data_ptr()), self._dt(q),
                                            ctypes.byref(st)))
        else:
            check(self.lib.mfa_schwarz_step(self.handle, None, MFA_F64, ctypes.byref(st)))
        return st.as_dict(self.degree)

    def fit_error(self):
        """(max |Q - N P|, ||Q - N P||_2) of the current control points against
        the data of the last encode or step (Algorithm 1's error vector)."""
        mx, l2 = c_double(0.0), c_double(0.0)
        check(self.lib.mfa_fit_error(self.handle, ctypes.byref(mx), ctypes.byref(l2)))
        return mx.value, l2.value

    def decode(self, out=None, dtype=None, deriv=None):
        torch = self.torch
        if out is None:
            out = torch.empty(self.npts, dtype=dtype or torch.float64, device=self.device)
        dt = self._check_out(out, self.npts)
        dptr = None
        if deriv is not None:
            arr = (c_int32 * 3)(*([int(r) for r in deriv] + [0] * (3 - len(deriv))))
            dptr = ctypes.cast(arr, POINTER(c_int32))
        check(self.lib.mfa_decode(self.handle, c_void_p(out.data_ptr()), dt, dptr))
        return out

    def decode_points(self, u, dtype=None, deriv=None, out=None):
        """Spline (or a mixed partial derivative) at parameter points u
        (npoints x dim float64 device tensor, values in [0, 1])."""
        torch = self.torch
        if u.dtype != torch.float64 or not u.is_contiguous() or u.dim() != 2 or \
                u.shape[1] != len(self.npts) or u.device != self.device:
            raise ValueError("u must be a contiguous (npoints, dim) float64 tensor on the device")
        npts = u.shape[0]
        if out is None:
            out = torch.empty(npts, dtype=dtype or torch.float64, device=self.device)
        dt = self._check_out(out, (npts,))
        dv = None
        if deriv is not None:
            dv = (c_int32 * len(deriv))(*[int(x) for x in deriv])
        check(self.lib.mfa_decode_points(self.handle, c_void_p(u.data_ptr()), npts,
                                         c_void_p(out.data_ptr()), dt, dv))
        return out

    def get_ctrl(self):
        torch = self.torch
        out = torch.empty(self.nctrl, dtype=torch.float64, device=self.device)
        check(self.lib.mfa_get_ctrl(self.handle, c_void_p(out.data_ptr()), 1))
        return out

    def warm_start(self):
        """The next encode starts from the control points the handle holds."""
        check(self.lib.mfa_set_ctrl(self.handle, None, 1))

    def set_stream(self, stream):
        """Enqueue this handle's later work on `stream` (a torch.cuda.Stream)."""
        check(self.lib.mfa_set_stream(self.handle, c_void_p(stream.cuda_stream)))
        self.stream = stream

    def set_ctrl(self, ctrl):
        if not isinstance(ctrl, self.torch.Tensor) or tuple(ctrl.shape) != self.nctrl or \
                ctrl.dtype != self.torch.float64 or ctrl.device != self.device:
            raise ValueError("control points must be a float64 tensor of shape %s on %s"
                             % (self.nctrl, self.device))
        src = ctrl.contiguous()
        check(self.lib.mfa_set_ctrl(self.handle, c_void_p(src.data_ptr()), 1))
        if src is not ctrl:
            # the copy is asynchronous on the handle's stream: keep the
            # temporary's memory from being reused before it has been read
            src.record_stream(self.stream)

    def set_timing(self, enable=True, classes=None, every=1, first=0):
        """Event-time the kernel classes named in `classes` (all when None):
        launches first, first + every, ... of each (all of them by default)."""
        mask = 0
        if enable:
            mask = 31 if classes is None else sum(1 << KERNEL_CLASSES[c] for c in classes)
        check(self.lib.mfa_set_timing_every(self.handle, int(every), int(first)))
        check(self.lib.mfa_set_timing(self.handle, mask))

    def kernel_time(self, kclass):
        """(total ms, launches) of one kernel class since the last read."""
        ms, n = c_double(0.0), c_int64(0)
        cid = KERNEL_CLASSES[kclass] if isinstance(kclass, str) else int(kclass)
        check(self.lib.mfa_kernel_time(self.handle, cid, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def inspect(self, table, axis=0, block=0):
        need = c_size_t(0)
        tid = TABLES[table] if isinstance(table, str) else int(table)
        check(self.lib.mfa_inspect(self.handle, tid, int(axis), int(block), None, 0,
                                   ctypes.byref(need)))
        buf = np.zeros(need.value, dtype=np.float64)
        check(self.lib.mfa_inspect(self.handle, tid, int(axis), int(block),
                                   buf.ctypes.data_as(POINTER(c_double)), buf.size, None))
        return buf
