"""ctypes binding of the C ABI in include/nmf.h (argument marshalling only).

Every step of the factorisation runs in the HIP library libnmf_hip.so; this
module only passes pointers and sizes.  PyTorch provides the device workspace
and the stream.  Importing works without a GPU; using a context needs one.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf_hip.so")

NMF_OK, NMF_CONVERGED = 0, 1
NMF_EINVAL, NMF_ENOMEM, NMF_EDEVICE, NMF_ENOTCONV = -1, -2, -3, -4
NMF_ESINGULAR, NMF_ESTATE, NMF_ECAPACITY = -5, -6, -7
GRAM_FP64, GRAM_FP32, GRAM_BF16X2 = 0, 1, 2

# Every symbol include/nmf.h declares.
EXPORTS = [
    "nmf_default_options", "nmf_workspace_bytes", "nmf_create", "nmf_anls_step", "nmf_ipm_step",
    "nmf_solve", "nmf_append_columns", "nmf_get_factors", "nmf_get_masks", "nmf_get_report",
    "nmf_get_shape", "nmf_destroy", "nmf_last_error", "nmf_status_string", "nmf_anls_profile",
    "nmf_get_duals", "nmf_set_launch_shape", "nmf_set_launch_fusion", "nmf_set_nnls_grouping", "nmf_set_ipm_precision", "nmf_get_launch_shape", "nmf_set_anls_budget", "nmf_batch_workspace_bytes", "nmf_batch_create",
    "nmf_batch_refresh", "nmf_batch_anls_step", "nmf_batch_poll", "nmf_batch_sync", "nmf_batch_destroy",
    "nmf_batch_create_static", "nmf_ipm_profile",
]
BATCH_STATIC_MAX = 1024   # NMF_BATCH_STATIC_MAX


class Options(ctypes.Structure):
    _fields_ = [
        ("eps_tol", ctypes.c_double), ("eps_stol", ctypes.c_double), ("tau", ctypes.c_double),
        ("eta", ctypes.c_double), ("sigma_c", ctypes.c_double), ("rho0_factor", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("inner_cap", ctypes.c_int32), ("exact_hessian_switch", ctypes.c_int32),
        ("max_anls_sweeps", ctypes.c_int32), ("max_ipm_iters", ctypes.c_int32),
        ("max_backtracks", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("gram_precision", ctypes.c_int32), ("with_ipm", ctypes.c_int32),
        ("x_splits", ctypes.c_int32), ("y_splits", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_double), ("E0", ctypes.c_double), ("Emu", ctypes.c_double),
        ("mu", ctypes.c_double), ("sigma", ctypes.c_double), ("step_rel", ctypes.c_double),
        ("stage", ctypes.c_int32), ("flag", ctypes.c_int32),
        ("sweeps", ctypes.c_int64), ("ipm_iters", ctypes.c_int64), ("ipm_outer", ctypes.c_int64),
        ("backtracks", ctypes.c_int64), ("nnls_solves", ctypes.c_int64), ("nnls_failed", ctypes.c_int64),
        ("mask_changes", ctypes.c_int64), ("exact_steps", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
        ("ms_stage1", ctypes.c_double), ("ms_stage2", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

# Live contexts and batches.  At interpreter exit they are released by
# _release_all() while torch's HIP runtime is still up (this handler is
# registered after torch is imported, so it runs before torch's own exit
# handlers); after that every __del__ is a no-op, so no HIP call is made
# while the runtime is being torn down.
_live_ctx = weakref.WeakSet()
_live_batch = weakref.WeakSet()
_exiting = False


def _release_all():
    global _exiting
    if _lib is None or _exiting:
        _exiting = True
        return
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for b in list(_live_batch):
        try:
            b.close()
        except Exception:
            pass
    for c in list(_live_ctx):
        try:
            c.close()
        except Exception:
            pass
    _exiting = True


def load():
    """Load libnmf_hip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (run paper_2101_08431_amd.build.build())")
    # PyTorch ships its own HIP runtime.  Importing it first makes this
    # library bind to that same runtime (the sonames match); loaded the other
    # way round, the process would hold two HIP runtimes and the second one
    # finds no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    atexit.register(_release_all)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.nmf_default_options.argtypes = [ctypes.POINTER(Options)]
    L.nmf_default_options.restype = None
    L.nmf_workspace_bytes.argtypes = [i64, i64, i32, ctypes.POINTER(Options)]
    L.nmf_workspace_bytes.restype = ctypes.c_size_t
    L.nmf_create.argtypes = [vp, i64, i64, i64, i32, i64, vp, vp, ctypes.POINTER(Options), vp,
                             ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.nmf_create.restype = ctypes.c_int
    for name in ("nmf_anls_step", "nmf_ipm_step"):
        getattr(L, name).argtypes = [vp, i32, ctypes.POINTER(Report)]
        getattr(L, name).restype = ctypes.c_int
    L.nmf_solve.argtypes = [vp, ctypes.POINTER(Report)]
    L.nmf_solve.restype = ctypes.c_int
    L.nmf_append_columns.argtypes = [vp, vp, i64, i64]
    L.nmf_append_columns.restype = ctypes.c_int
    L.nmf_get_factors.argtypes = [vp, vp, vp]
    L.nmf_get_factors.restype = ctypes.c_int
    L.nmf_get_duals.argtypes = [vp, vp, vp]
    L.nmf_get_duals.restype = ctypes.c_int
    L.nmf_get_masks.argtypes = [vp, vp, vp]
    L.nmf_get_masks.restype = ctypes.c_int
    L.nmf_get_report.argtypes = [vp, ctypes.POINTER(Report)]
    L.nmf_get_report.restype = ctypes.c_int
    L.nmf_anls_profile.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.nmf_anls_profile.restype = ctypes.c_int
    L.nmf_ipm_profile.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.nmf_ipm_profile.restype = ctypes.c_int
    L.nmf_set_launch_shape.argtypes = [vp, i32, i32]
    L.nmf_set_launch_shape.restype = ctypes.c_int
    L.nmf_set_launch_fusion.argtypes = [vp, i32, i32]
    L.nmf_set_launch_fusion.restype = ctypes.c_int
    L.nmf_set_nnls_grouping.argtypes = [vp, i32]
    L.nmf_set_nnls_grouping.restype = ctypes.c_int
    L.nmf_set_ipm_precision.argtypes = [vp, i32, i32]
    L.nmf_set_ipm_precision.restype = ctypes.c_int
    L.nmf_get_launch_shape.argtypes = [vp, vp]
    L.nmf_get_launch_shape.restype = ctypes.c_int
    L.nmf_set_anls_budget.argtypes = [vp, i32]
    L.nmf_set_anls_budget.restype = ctypes.c_int
    L.nmf_batch_workspace_bytes.argtypes = [i32]
    L.nmf_batch_workspace_bytes.restype = ctypes.c_size_t
    L.nmf_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.nmf_batch_create.restype = ctypes.c_int
    L.nmf_batch_create_static.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(vp)]
    L.nmf_batch_create_static.restype = ctypes.c_int
    for name in ("nmf_batch_refresh", "nmf_batch_sync", "nmf_batch_destroy"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = ctypes.c_int
    L.nmf_batch_anls_step.argtypes = [vp, i32, i32]
    L.nmf_batch_anls_step.restype = ctypes.c_int
    L.nmf_batch_poll.argtypes = [vp, vp, vp]
    L.nmf_batch_poll.restype = ctypes.c_int
    L.nmf_get_shape.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.nmf_get_shape.restype = ctypes.c_int
    L.nmf_destroy.argtypes = [vp]
    L.nmf_destroy.restype = ctypes.c_int
    L.nmf_last_error.argtypes = [vp]
    L.nmf_last_error.restype = ctypes.c_char_p
    L.nmf_status_string.argtypes = [ctypes.c_int]
    L.nmf_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def default_options(**kw):
    o = Options()
    load().nmf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def workspace_bytes(n, m_capacity, k, opts=None):
    o = opts if opts is not None else default_options()
    return int(load().nmf_workspace_bytes(int(n), int(m_capacity), int(k), ctypes.byref(o)))


class NMFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{load().nmf_status_string(status).decode()}: {msg}")
        self.status = status


def _ptr(a):
    """Device or host address of a torch tensor or numpy array (contiguous)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr())
    if not a.flags["C_CONTIGUOUS"] and not a.flags["F_CONTIGUOUS"]:
        raise ValueError("array must be contiguous")
    return ctypes.c_void_p(a.ctypes.data)


class NMF:
    """One streaming factorisation living in a device workspace.

    M: (n, m) float64, column-major host array (numpy, Fortran order) or a
    torch tensor of shape (m, n) on the GPU (its rows are the columns of M).
    X0: (n, k) row-major; Y0: (k, m) row-major; numpy or torch (host or GPU).
    """

    def __init__(self, M, k, X0=None, Y0=None, m_capacity=None, options=None, stream=None, device=None):
        import torch
        L = load()
        self._torch = torch
        if hasattr(M, "data_ptr"):
            m, n = M.shape
            Mptr, ldm = _ptr(M), n
        else:
            n, m = M.shape
            if not M.flags["F_CONTIGUOUS"]:
                raise ValueError("host M must be column-major (numpy Fortran order)")
            Mptr, ldm = _ptr(M), n
        self._keep = [M, X0, Y0]
        self.options = options if options is not None else default_options()
        cap = int(m_capacity) if m_capacity is not None else int(m)
        nbytes = workspace_bytes(n, cap, k, self.options)
        if nbytes == 0:
            raise NMFError(NMF_EINVAL, "invalid sizes")
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        out = ctypes.c_void_p()
        st = L.nmf_create(Mptr, n, m, ldm, int(k), cap, _ptr(X0), _ptr(Y0), ctypes.byref(self.options),
                          ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out))
        if st != NMF_OK:
            raise NMFError(st, L.nmf_last_error(None).decode())
        self._ctx = out
        self.n, self.k = int(n), int(k)
        _live_ctx.add(self)

    # -- helpers
    def _check(self, st, ok=(NMF_OK, NMF_CONVERGED, NMF_ENOTCONV)):
        if st not in ok:
            raise NMFError(st, load().nmf_last_error(self._ctx).decode())
        return st

    @property
    def m(self):
        n, m, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        load().nmf_get_shape(self._ctx, ctypes.byref(n), ctypes.byref(m), ctypes.byref(k))
        return int(m.value)

    def anls_step(self, sweeps, report=True):
        r = Report() if report else None
        st = self._check(load().nmf_anls_step(self._ctx, int(sweeps), ctypes.byref(r) if r else None))
        return (st, r.as_dict()) if r is not None else st

    def ipm_step(self, iters, report=True):
        r = Report() if report else None
        st = self._check(load().nmf_ipm_step(self._ctx, int(iters), ctypes.byref(r) if r else None))
        return (st, r.as_dict()) if r is not None else st

    def anls_profile(self, sweeps):
        """Mean device ms of the four stage-1 kernels over `sweeps` sweeps:
        (x stream, row NNLS, y stream, column NNLS)."""
        ms = (ctypes.c_double * 4)()
        self._check(load().nmf_anls_profile(self._ctx, int(sweeps), ms), ok=(NMF_OK,))
        return tuple(ms)

    def ipm_profile(self, iters):
        """Runs up to `iters` stage-2 inner iterations with the dense steps
        event-timed.  Returns (status, ms, counts): ms = mean device ms of a
        Gauss-Newton Schur formation, an exact-Hessian formation, a Cholesky
        factorisation, a pair of triangular solves, and wall ms per inner
        iteration; counts = how many of each (the last: inner iterations)."""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int64 * 5)()
        st = self._check(load().nmf_ipm_profile(self._ctx, int(iters), ms, cnt))
        return st, tuple(ms), tuple(int(v) for v in cnt)

    def solve(self):
        r = Report()
        st = self._check(load().nmf_solve(self._ctx, ctypes.byref(r)))
        return st, r.as_dict()

    def report(self):
        r = Report()
        self._check(load().nmf_get_report(self._ctx, ctypes.byref(r)))
        return r.as_dict()

    def append_columns(self, Mnew):
        if hasattr(Mnew, "data_ptr"):
            mnew, n = Mnew.shape
        else:
            n, mnew = Mnew.shape
            if not Mnew.flags["F_CONTIGUOUS"]:
                raise ValueError("host columns must be column-major")
        if n != self.n:
            raise ValueError("row count differs")
        self._keep.append(Mnew)
        self._check(load().nmf_append_columns(self._ctx, _ptr(Mnew), int(mnew), int(n)), ok=(NMF_OK,))

    def factors(self):
        """(X (n, k), Y (k, m)) as host numpy float64 arrays."""
        import numpy as np
        X = np.empty((self.n, self.k))
        Y = np.empty((self.k, self.m))
        self._check(load().nmf_get_factors(self._ctx, _ptr(X), _ptr(Y)), ok=(NMF_OK,))
        return X, Y

    def duals(self):
        """Stage-2 duals (R (n, k), S (k, m)) as host numpy arrays."""
        import numpy as np
        R = np.empty((self.n, self.k))
        S = np.empty((self.k, self.m))
        self._check(load().nmf_get_duals(self._ctx, _ptr(R), _ptr(S)), ok=(NMF_OK,))
        return R, S

    def masks(self):
        import numpy as np
        xm = np.empty(self.n, dtype=np.uint32)
        ym = np.empty(self.m, dtype=np.uint32)
        self._check(load().nmf_get_masks(self._ctx, _ptr(xm), _ptr(ym)), ok=(NMF_OK,))
        return xm, ym

    def set_anls_budget(self, max_sweeps):
        """Stage-1 sweep budget from now on (re-arms the stop rule)."""
        self._check(load().nmf_set_anls_budget(self._ctx, int(max_sweeps)), ok=(NMF_OK,))

    def set_launch_shape(self, x_splits, y_splits):
        self._check(load().nmf_set_launch_shape(self._ctx, int(x_splits), int(y_splits)), ok=(NMF_OK,))

    def set_launch_fusion(self, fuse_x, fuse_y):
        """1: the half is one kernel (the tile's last split solves), 0: stream +
        NNLS kernels, -1: one kernel exactly when the half has a single split."""
        self._check(load().nmf_set_launch_fusion(self._ctx, int(fuse_x), int(fuse_y)), ok=(NMF_OK,))

    def set_ipm_precision(self, mixed, refine_steps=2):
        """1: exact-Hessian Schur formation in FP32 with FP64 refinement of the
        direction; 0: FP64 throughout."""
        self._check(load().nmf_set_ipm_precision(self._ctx, int(mixed), int(refine_steps)), ok=(NMF_OK,))

    def set_nnls_grouping(self, on):
        """1: passive-set-grouped first solves in the stage-1 halves (one
        (G_PP)^-1 per distinct warm-start set), 0: the per-problem loop."""
        self._check(load().nmf_set_nnls_grouping(self._ctx, int(on)), ok=(NMF_OK,))

    def launch_plan(self):
        """(x splits, y splits, X-half one kernel, Y-half one kernel) in effect."""
        out = (ctypes.c_int32 * 4)()
        self._check(load().nmf_get_launch_shape(self._ctx, out), ok=(NMF_OK,))
        return int(out[0]), int(out[1]), bool(out[2]), bool(out[3])

    def close(self):
        """Releases the context now (its workspace is freed with this object)."""
        if getattr(self, "_ctx", None):
            load().nmf_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        if _exiting or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Stage-1 sweeps of many contexts in shared launches (see nmf_batch_* in
    include/nmf.h).  Uses its own non-default stream so sweeps can be captured
    into a HIP graph."""

    def __init__(self, contexts, stream=None, static=False):
        """static=True builds the batch with nmf_batch_create_static: no
        workspace is allocated (the library's own per-device table array is
        used, so only the most recent static batch is valid)."""
        import torch
        L = load()
        self.contexts = list(contexts)
        n = len(self.contexts)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        arr = (ctypes.c_void_p * n)(*[c._ctx.value for c in self.contexts])
        out = ctypes.c_void_p()
        # the contexts' setup work runs on their own streams
        for c in self.contexts:
            c.stream.synchronize()
        if static:
            self.workspace = None
            st = L.nmf_batch_create_static(arr, n, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out))
        else:
            nbytes = int(L.nmf_batch_workspace_bytes(n))
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            st = L.nmf_batch_create(arr, n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out))
        if st != NMF_OK:
            raise NMFError(st, L.nmf_last_error(None).decode())
        self._b = out
        _live_batch.add(self)

    def step(self, sweeps, graph=True):
        st = load().nmf_batch_anls_step(self._b, int(sweeps), 1 if graph else 0)
        if st != NMF_OK:
            raise NMFError(st, "batched sweep failed")

    def refresh(self):
        st = load().nmf_batch_refresh(self._b)
        if st != NMF_OK:
            raise NMFError(st, "batch refresh failed")

    def sync(self):
        load().nmf_batch_sync(self._b)

    def poll(self):
        """Waits for the batch, then returns (converged, sweeps): numpy arrays
        over the contexts in the order given at construction."""
        import numpy as np
        n = len(self.contexts)
        conv = np.zeros(n, dtype=np.int32)
        sw = np.zeros(n, dtype=np.int64)
        st = load().nmf_batch_poll(self._b, _ptr(conv), _ptr(sw))
        if st != NMF_OK:
            raise NMFError(st, "batch poll failed")
        return conv.astype(bool), sw

    def close(self):
        """Waits for the batch's stream, then releases the batch and its graph."""
        if getattr(self, "_b", None):
            load().nmf_batch_sync(self._b)
            load().nmf_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        if _exiting or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
