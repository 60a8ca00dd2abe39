"""ctypes binding of libtvdeblur.so (include/tvdeblur.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Images are torch tensors on the HIP device (float64 for the
'f64' precision, float32 for 'f32_mixed'); work is queued on torch's current
stream of that device.  The binding raises if the library is not built --
there is no CPU fallback.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtvdeblur.so")

TVD_OK = 0
ERRORS = {-1: "TVD_EINVAL", -2: "TVD_ENOTSYM", -3: "TVD_ENORM", -4: "TVD_ESIZE", -5: "TVD_ESTATE",
          -6: "TVD_EDEVICE", -7: "TVD_EBREAKDOWN", -8: "TVD_ENOMEM"}
PRECISION = {"f64": 0, "f32_mixed": 1}
BC = {"reflective": 1, "antireflective": 2, "dirichlet": 3, "periodic": 4}
PRECOND = {"none": 0, "diag": 1, "x": 2, "d_x": 3, "x_d": 4}
# preconditioners of the reblurring system: I, D and P, D_P, P_D (Section 3)
# on the same enum slots
REBLUR_PRECOND = {"none": 0, "diag": 1, "p": 2, "d_p": 3, "p_d": 4}
EXPORT = {"kappa": 0, "s": 1, "mu": 2, "lambda_h": 3, "d": 4}
MAX_OUTER = 256
KTIME_KINDS = 12
TRANSFORM = {"auto": 0, "fft": 1, "gemm": 2}

# Every symbol declared in include/tvdeblur.h.
EXPORTED_SYMBOLS = (
    "tvdeblur_create", "tvdeblur_set_psf", "tvdeblur_set_bc", "tvdeblur_solve", "tvdeblur_destroy",
    "tvdeblur_last_error", "tvdeblur_op_blur", "tvdeblur_op_blur_adjoint", "tvdeblur_op_setup",
    "tvdeblur_op_normal", "tvdeblur_op_precond", "tvdeblur_op_export", "tvdeblur_set_profiling",
    "tvdeblur_get_kernel_times", "tvdeblur_solve_adjoint", "tvdeblur_batch_create", "tvdeblur_batch_solve",
    "tvdeblur_batch_get_info", "tvdeblur_batch_destroy", "tvdeblur_batch_last_error",
    "tvdeblur_set_transform", "tvdeblur_get_transform", "tvdeblur_time_kernel",
    "tvdeblur_solve_reblur", "tvdeblur_op_reblur_setup", "tvdeblur_op_reblur_normal",
    "tvdeblur_op_reblur_precond", "tvdeblur_solve_noalloc", "tvdeblur_signals_create", "tvdeblur_signals_solve",
    "tvdeblur_signals_destroy", "tvdeblur_signals_last_error", "tvdeblur_set_reblur_l_bc",
    "tvdeblur_workspace_bytes", "tvdeblur_set_workspace", "tvdeblur_get_gemm_tile",
    "tvdeblur_set_gemm_tile",
)
BATCH_PRECOND = ("x", "d_x", "x_d")


class TvdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("fp_tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("max_inner", ctypes.c_int),
                ("precond", ctypes.c_int), ("u0_dev", ctypes.c_void_p), ("replay_host", ctypes.POINTER(ctypes.c_int)),
                ("iterates_dev", ctypes.c_void_p), ("record_objective", ctypes.c_int), ("use_graph", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_steps", ctypes.c_int), ("inner_iters", ctypes.c_int * MAX_OUTER),
                ("relres", ctypes.c_double * MAX_OUTER), ("fp_change", ctypes.c_double * MAX_OUTER),
                ("all_converged", ctypes.c_int), ("breakdown", ctypes.c_int),
                ("total_inner_iters", ctypes.c_longlong), ("time_total_s", ctypes.c_double),
                ("time_setup_s", ctypes.c_double), ("time_inner_s", ctypes.c_double),
                ("tv_objective", ctypes.c_double * (MAX_OUTER + 1))]

    def to_dict(self):
        k = self.outer_steps
        return {"outer_steps": k, "inner_iters": list(self.inner_iters[:k]), "relres": list(self.relres[:k]),
                "tv_objective": list(self.tv_objective[:k + 1]),
                "fp_change": list(self.fp_change[:k]), "all_converged": bool(self.all_converged),
                "breakdown": bool(self.breakdown), "total_inner_iters": int(self.total_inner_iters),
                "time_total_s": self.time_total_s, "time_setup_s": self.time_setup_s,
                "time_inner_s": self.time_inner_s}


class KernelTimes(ctypes.Structure):
    _fields_ = [("n_kinds", ctypes.c_int), ("name", (ctypes.c_char * 24) * KTIME_KINDS),
                ("launches", ctypes.c_longlong * KTIME_KINDS), ("total_ms", ctypes.c_double * KTIME_KINDS)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int), ("nx", ctypes.c_int), ("psf_host", ctypes.POINTER(ctypes.c_double)),
                ("py", ctypes.c_int), ("px", ctypes.c_int)]


class BatchParams(ctypes.Structure):
    _fields_ = [("alpha_host", ctypes.POINTER(ctypes.c_double)), ("beta_host", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.c_double), ("max_outer", ctypes.c_int), ("fp_tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("max_inner", ctypes.c_int), ("precond", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("replay_host", ctypes.POINTER(ctypes.c_int)),
                ("transform", ctypes.c_int), ("gemm_tile", ctypes.c_int)]


TUNE_MAX = 4


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("line_threads", ctypes.c_int), ("tables_in_lds", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("n_candidates", ctypes.c_int),
                ("cand_threads", ctypes.c_int * TUNE_MAX), ("cand_us", ctypes.c_double * TUNE_MAX),
                ("gemm_us", ctypes.c_double), ("transform", ctypes.c_int),
                ("graph_launches", ctypes.c_longlong), ("time_setup_s", ctypes.c_double),
                ("time_inner_s", ctypes.c_double), ("gemm64_us", ctypes.c_double), ("gemm_tile", ctypes.c_int)]


class SignalDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("psf_host", ctypes.POINTER(ctypes.c_double)), ("plen", ctypes.c_int),
                ("bc", ctypes.c_int), ("reblur", ctypes.c_int)]


class SignalParams(ctypes.Structure):
    _fields_ = [("alpha_host", ctypes.POINTER(ctypes.c_double)), ("beta_host", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.c_double), ("precond_host", ctypes.POINTER(ctypes.c_int)), ("precond", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("fp_tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("max_inner", ctypes.c_int), ("replay_host", ctypes.POINTER(ctypes.c_int)),
                ("system_host", ctypes.POINTER(ctypes.c_int)), ("system", ctypes.c_int)]


_lib = None


def load():
    """Load libtvdeblur.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1011_5964_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "tvdeblur_create": [ctypes.POINTER(vp), i, i, i, vp],
        "tvdeblur_set_psf": [vp, ctypes.POINTER(d), i, i],
        "tvdeblur_set_bc": [vp, i],
        "tvdeblur_solve": [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Stats)],
        "tvdeblur_solve_noalloc": [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Stats)],
        "tvdeblur_destroy": [vp],
        "tvdeblur_op_blur": [vp, vp, vp],
        "tvdeblur_op_blur_adjoint": [vp, vp, vp],
        "tvdeblur_op_setup": [vp, vp, d, d, i],
        "tvdeblur_op_normal": [vp, vp, vp],
        "tvdeblur_op_precond": [vp, vp, vp],
        "tvdeblur_solve_reblur": [vp, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(Stats)],
        "tvdeblur_op_reblur_setup": [vp, vp, d, d, i],
        "tvdeblur_op_reblur_normal": [vp, vp, vp],
        "tvdeblur_op_reblur_precond": [vp, vp, vp],
        "tvdeblur_op_export": [vp, i, vp],
        "tvdeblur_set_profiling": [vp, i],
        "tvdeblur_get_kernel_times": [vp, ctypes.POINTER(KernelTimes)],
        "tvdeblur_time_kernel": [vp, i, i, ctypes.POINTER(ctypes.c_double)],
        "tvdeblur_solve_adjoint": [vp, vp, i, vp, vp, ctypes.POINTER(d), ctypes.POINTER(d),
                                   ctypes.POINTER(Params), ctypes.POINTER(Stats)],
        "tvdeblur_batch_create": [ctypes.POINTER(vp), i, ctypes.POINTER(ImageDesc), i, i, vp],
        "tvdeblur_batch_solve": [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(BatchParams),
                                 ctypes.POINTER(Stats)],
        "tvdeblur_batch_get_info": [vp, ctypes.POINTER(BatchInfo)],
        "tvdeblur_batch_destroy": [vp],
        "tvdeblur_set_transform": [vp, i],
        "tvdeblur_get_transform": [vp, ctypes.POINTER(i)],
        "tvdeblur_signals_create": [ctypes.POINTER(vp), i, ctypes.POINTER(SignalDesc), vp],
        "tvdeblur_signals_solve": [vp, vp, vp, ctypes.POINTER(SignalParams), ctypes.POINTER(Stats)],
        "tvdeblur_signals_destroy": [vp],
        "tvdeblur_set_reblur_l_bc": [vp, i],
        "tvdeblur_workspace_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "tvdeblur_set_workspace": [vp, vp, ctypes.c_size_t],
        "tvdeblur_get_gemm_tile": [vp, ctypes.POINTER(i)],
        "tvdeblur_set_gemm_tile": [vp, i],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i
    for name in ("tvdeblur_last_error", "tvdeblur_batch_last_error", "tvdeblur_signals_last_error"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class TVDeblur:
    """One handle: fixed image shape, precision and stream."""

    def __init__(self, ny, nx, precision="f32_mixed", stream=None):
        import torch
        self.lib = load()
        self.ny, self.nx = int(ny), int(nx)
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = stream.device
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_create(ctypes.byref(h), self.ny, self.nx, PRECISION[precision],
                                          ctypes.c_void_p(stream.cuda_stream))
        if rc != TVD_OK:
            raise TvdError(rc, self.lib.tvdeblur_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != TVD_OK:
            raise TvdError(rc, self.lib.tvdeblur_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tvdeblur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, t, name):
        if t.dtype != self.dtype or tuple(t.shape) != (self.ny, self.nx) or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} ({self.ny}, {self.nx}) tensor on {self.device}")
        return t

    def set_psf(self, psf):
        h = np.ascontiguousarray(psf, dtype=np.float64)
        self._check(self.lib.tvdeblur_set_psf(self.h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              h.shape[0], h.shape[1]))

    def set_bc(self, bc):
        self._check(self.lib.tvdeblur_set_bc(self.h, BC[bc]))

    def _params(self, alpha, beta, max_outer, inner_tol, max_inner, precond_code, fp_tol, u0, replay, iterates,
                objective=False, use_graph=False):
        p = Params()
        p.record_objective = 1 if objective else 0
        p.use_graph = 1 if use_graph else 0
        p.alpha, p.beta, p.max_outer = float(alpha), float(beta), int(max_outer)
        p.fp_tol, p.inner_tol, p.max_inner = float(fp_tol), float(inner_tol), int(max_inner)
        p.precond = precond_code
        p.u0_dev = None if u0 is None else self._img(u0, "u0").data_ptr()
        keep = None
        if replay is not None:
            # the library reads max_outer counts from this array
            if len(replay) < int(max_outer):
                raise ValueError(f"replay needs max_outer = {int(max_outer)} counts, got {len(replay)}")
            keep = (ctypes.c_int * len(replay))(*[int(x) for x in replay])
            p.replay_host = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int))
        if iterates is not None:
            if iterates.dtype != self.dtype or not iterates.is_contiguous() or iterates.device != self.device \
                    or iterates.numel() < (max_outer + 1) * self.ny * self.nx:
                raise ValueError(f"iterates must be a contiguous {self.dtype} tensor on {self.device} "
                                 f"holding max_outer + 1 images")
            p.iterates_dev = iterates.data_ptr()
        return p, keep

    def solve(self, v, alpha, beta, max_outer, inner_tol=1e-6, max_inner=100, precond="x_d", fp_tol=0.0,
              u0=None, replay=None, iterates=None, out=None, objective=False, use_graph=False):
        """objective: also return T(u^0..u^K) of eq. (mp) in stats['tv_objective'].
        use_graph: replay the PCG iterations from HIP graphs (same bits)."""
        import torch
        self._img(v, "v")
        u = self._img(out, "out") if out is not None else torch.empty_like(v)
        p, keep = self._params(alpha, beta, max_outer, inner_tol, max_inner, PRECOND[precond], fp_tol, u0,
                               replay, iterates, objective, use_graph)
        st = Stats()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_solve(self.h, _ptr(v), _ptr(u), ctypes.byref(p), ctypes.byref(st))
        del keep
        self._check(rc)
        return u, st.to_dict()

    def solve_noalloc(self, v, out, alpha, beta, max_outer, inner_tol=1e-6, max_inner=100, precond="x_d",
                      fp_tol=0.0, u0=None, replay=None, iterates=None):
        """tvdeblur_solve_noalloc: as solve, writing the caller's `out`, with
        the work buffers in the library's static device array (the handle
        must be built: call transform() once first)."""
        self._img(v, "v")
        self._img(out, "out")
        p, keep = self._params(alpha, beta, max_outer, inner_tol, max_inner, PRECOND[precond], fp_tol, u0,
                               replay, iterates)
        st = Stats()
        import torch
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_solve_noalloc(self.h, _ptr(v), _ptr(out), ctypes.byref(p), ctypes.byref(st))
        del keep
        self._check(rc)
        return out, st.to_dict()

    def workspace_bytes(self):
        """tvdeblur_workspace_bytes: bytes of a caller-owned work area for
        solve (builds the handle for its PSF and BC)."""
        n = ctypes.c_size_t(0)
        self._check(self.lib.tvdeblur_workspace_bytes(self.h, ctypes.byref(n)))
        return n.value

    def set_workspace(self, ws):
        """tvdeblur_set_workspace: solve carves its work buffers from `ws`
        (a contiguous device tensor of at least workspace_bytes() bytes,
        256-byte aligned); None returns to the handle's own.  The handle
        keeps a reference to `ws` while it is set."""
        if ws is None:
            self._check(self.lib.tvdeblur_set_workspace(self.h, None, 0))
            self._ws = None
            return
        if not ws.is_cuda or not ws.is_contiguous() or ws.device != self.device:
            raise ValueError(f"workspace must be a contiguous tensor on {self.device}")
        self._check(self.lib.tvdeblur_set_workspace(self.h, _ptr(ws), ws.numel() * ws.element_size()))
        self._ws = ws

    def set_reblur_l_bc(self, l_bc):
        """BC of L(u^k) in the reblurring system: 'neumann' (default) or
        'antireflective'."""
        self._check(self.lib.tvdeblur_set_reblur_l_bc(self.h, {"neumann": 0, "antireflective": 2}[l_bc]))

    def solve_reblur(self, v, alpha, beta, max_outer, inner_tol=1e-6, max_inner=100, precond="p_d", fp_tol=0.0,
                     u0=None, replay=None, iterates=None, out=None):
        """The reblurring system (H'H + alpha L(u^k)) u^{k+1} = H'v by
        PBiCGstab with I, D, P, D_P or P_D ('none', 'diag', 'p', 'd_p',
        'p_d'); see
        tvdeblur_solve_reblur.  inner_iters counts BiCGstab iterations."""
        import torch
        self._img(v, "v")
        if precond not in REBLUR_PRECOND:
            raise ValueError(f"precond must be one of {sorted(REBLUR_PRECOND)}")
        u = self._img(out, "out") if out is not None else torch.empty_like(v)
        p, keep = self._params(alpha, beta, max_outer, inner_tol, max_inner, REBLUR_PRECOND[precond], fp_tol, u0,
                               replay, iterates)
        st = Stats()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_solve_reblur(self.h, _ptr(v), _ptr(u), ctypes.byref(p), ctypes.byref(st))
        del keep
        self._check(rc)
        return u, st.to_dict()

    def solve_adjoint(self, iterates, K, ubar, alpha, beta, inner_tol=1e-6, max_inner=100, precond="x_d"):
        """Gradients (vbar, alphabar, betabar, stats) of a loss with dl/du^K =
        ubar, through the K fixed-point steps whose iterates u^0..u^K are in
        `iterates` (as filled by solve(..., iterates=...))."""
        import torch
        self._img(ubar, "ubar")
        if iterates.dtype != self.dtype or not iterates.is_contiguous() or \
                iterates.numel() < (K + 1) * self.ny * self.nx:
            raise ValueError("iterates must hold K+1 contiguous images of the handle's type")
        vbar = torch.empty_like(ubar)
        p = Params()
        p.alpha, p.beta, p.max_outer = float(alpha), float(beta), int(K)
        p.inner_tol, p.max_inner, p.precond = float(inner_tol), int(max_inner), PRECOND[precond]
        ab, bb = ctypes.c_double(), ctypes.c_double()
        st = Stats()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_solve_adjoint(self.h, ctypes.c_void_p(iterates.data_ptr()), int(K), _ptr(ubar),
                                                 _ptr(vbar), ctypes.byref(ab), ctypes.byref(bb), ctypes.byref(p),
                                                 ctypes.byref(st))
        self._check(rc)
        return vbar, ab.value, bb.value, st.to_dict()

    def set_transform(self, mode):
        """'auto' (pick the faster at build), 'fft' or 'gemm' (see tvdeblur_set_transform)."""
        self._check(self.lib.tvdeblur_set_transform(self.h, TRANSFORM[mode]))

    def transform(self):
        """The transform implementation in use: 'fft' or 'gemm'."""
        v = ctypes.c_int()
        self._check(self.lib.tvdeblur_get_transform(self.h, ctypes.byref(v)))
        return {1: "fft", 2: "gemm"}[v.value]

    def set_gemm_tile(self, tile):
        """Block tile of the products: 0 (timed at build), 32 or 64."""
        self._check(self.lib.tvdeblur_set_gemm_tile(self.h, int(tile)))

    def gemm_tile(self):
        """Block tile of the matrix-core products (32 or 64), timed at build."""
        v = ctypes.c_int()
        self._check(self.lib.tvdeblur_get_gemm_tile(self.h, ctypes.byref(v)))
        return v.value

    def set_profiling(self, every):
        """every: time every every-th launch of each kernel class (True = 1);
        0 / False stops."""
        self._check(self.lib.tvdeblur_set_profiling(self.h, int(every)))

    def kernel_times(self):
        kt = KernelTimes()
        self._check(self.lib.tvdeblur_get_kernel_times(self.h, ctypes.byref(kt)))
        return {kt.name[k].value.decode(): {"launches": int(kt.launches[k]), "total_ms": float(kt.total_ms[k])}
                for k in range(kt.n_kinds)}

    def time_kernel(self, kind, reps=50):
        """Average duration in microseconds of one launch of a PCG-loop kernel
        class ('band_normal', 'column', 'update', 'transform_gemm' or 'x_pass'), from a
        back-to-back burst of reps launches with the parameters of the last
        solve (see tvdeblur_time_kernel)."""
        kinds = {"band_normal": 0, "column": 2, "update": 7, "transform_gemm": 8, "x_pass": 9}
        if kind not in kinds:
            raise ValueError(f"kind must be one of {sorted(kinds)}")
        import torch
        out = ctypes.c_double()
        with torch.cuda.device(self.device):
            self._check(self.lib.tvdeblur_time_kernel(self.h, kinds[kind], int(reps), ctypes.byref(out)))
        return out.value

    # single operators
    def _op(self, fn, x, name):
        import torch
        self._img(x, name)
        y = torch.empty_like(x)
        with torch.cuda.device(self.device):
            self._check(fn(self.h, _ptr(x), _ptr(y)))
        return y

    def blur(self, x):
        return self._op(self.lib.tvdeblur_op_blur, x, "x")

    def blur_adjoint(self, x):
        return self._op(self.lib.tvdeblur_op_blur_adjoint, x, "x")

    def setup(self, uk, alpha, beta, precond="x_d"):
        import torch
        self._img(uk, "uk")
        with torch.cuda.device(self.device):
            self._check(self.lib.tvdeblur_op_setup(self.h, _ptr(uk), float(alpha), float(beta), PRECOND[precond]))

    def normal(self, x):
        return self._op(self.lib.tvdeblur_op_normal, x, "x")

    def reblur_setup(self, uk, alpha, beta, precond="p_d"):
        import torch
        self._img(uk, "uk")
        if precond not in REBLUR_PRECOND:
            raise ValueError(f"precond must be one of {sorted(REBLUR_PRECOND)}")
        with torch.cuda.device(self.device):
            self._check(self.lib.tvdeblur_op_reblur_setup(self.h, _ptr(uk), float(alpha), float(beta),
                                                          REBLUR_PRECOND[precond]))

    def reblur_normal(self, x):
        return self._op(self.lib.tvdeblur_op_reblur_normal, x, "x")

    def reblur_precond(self, r):
        return self._op(self.lib.tvdeblur_op_reblur_precond, r, "r")

    def precond(self, r):
        return self._op(self.lib.tvdeblur_op_precond, r, "r")

    def export(self, which):
        import torch
        out = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._check(self.lib.tvdeblur_op_export(self.h, EXPORT[which], _ptr(out)))
        return out


class TVDeblurBatch:
    """Batching form: independent images of different sizes, each with its
    own PSF, alpha and beta, solved together (one launch per PCG stage for
    the whole batch).  shapes: list of (ny, nx); psfs: list of 2D arrays."""

    def __init__(self, shapes, psfs, bc, precision="f32_mixed", stream=None):
        import torch
        if len(shapes) != len(psfs) or not shapes:
            raise ValueError("shapes and psfs must be non-empty lists of the same length")
        self.lib = load()
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        self.count = len(self.shapes)
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.device = stream.device
        self._psfs = [np.ascontiguousarray(h, dtype=np.float64) for h in psfs]
        descs = (ImageDesc * self.count)()
        for k, ((ny, nx), h) in enumerate(zip(self.shapes, self._psfs)):
            descs[k] = ImageDesc(ny, nx, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), h.shape[0], h.shape[1])
        b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_batch_create(ctypes.byref(b), self.count, descs, PRECISION[precision], BC[bc],
                                                ctypes.c_void_p(stream.cuda_stream))
        if rc != TVD_OK:
            raise TvdError(rc, self.lib.tvdeblur_batch_last_error(None).decode())
        self.b = b

    def _check(self, rc):
        if rc != TVD_OK:
            raise TvdError(rc, self.lib.tvdeblur_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None):
            self.lib.tvdeblur_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, vs, alphas, beta=0.05, betas=None, max_outer=10, inner_tol=1e-6, max_inner=100,
              precond="x_d", fp_tol=0.0, use_graph=True, outs=None, replay=None, transform="auto", gemm_tile=0):
        """Returns (list of restored images, list of per-image stats dicts).
        replay: None, or per image a list of max_outer PCG iteration counts.
        transform: 'auto' (the implementation picked at create), 'fft' or 'gemm'.
        gemm_tile: block tile of the products, 0 (picked at create), 32 or 64."""
        import torch
        if len(vs) != self.count or len(alphas) != self.count:
            raise ValueError("one v and one alpha per image")
        for k, v in enumerate(vs):
            if v.dtype != self.dtype or tuple(v.shape) != self.shapes[k] or not v.is_contiguous() \
                    or v.device != self.device:
                raise ValueError(f"v[{k}] must be a contiguous {self.dtype} {self.shapes[k]} tensor on {self.device}")
        if outs is not None:
            if len(outs) != self.count:
                raise ValueError("one output per image")
            for k, u in enumerate(outs):
                if u.dtype != self.dtype or tuple(u.shape) != self.shapes[k] or not u.is_contiguous() \
                        or u.device != self.device:
                    raise ValueError(f"outs[{k}] must be a contiguous {self.dtype} {self.shapes[k]} tensor "
                                     f"on {self.device}")
        us = outs if outs is not None else [torch.empty_like(v) for v in vs]
        vp = (ctypes.c_void_p * self.count)(*[v.data_ptr() for v in vs])
        up = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in us])
        a = (ctypes.c_double * self.count)(*[float(x) for x in alphas])
        p = BatchParams()
        p.alpha_host = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        bkeep = None
        if betas is not None:
            bkeep = (ctypes.c_double * self.count)(*[float(x) for x in betas])
            p.beta_host = ctypes.cast(bkeep, ctypes.POINTER(ctypes.c_double))
        p.beta, p.max_outer, p.fp_tol = float(beta), int(max_outer), float(fp_tol)
        p.inner_tol, p.max_inner, p.precond = float(inner_tol), int(max_inner), PRECOND[precond]
        p.use_graph = 1 if use_graph else 0
        p.transform = TRANSFORM[transform]
        p.gemm_tile = int(gemm_tile)
        rkeep = None
        if replay is not None:
            # count x max_outer counts, image-major, read in full by the library;
            # a shorter list (an image that stops early on fp_tol) is padded with zeros
            if len(replay) != self.count or any(len(r) > int(max_outer) for r in replay):
                raise ValueError(f"replay needs {self.count} lists of at most max_outer = {int(max_outer)} counts")
            flat = [int(c) for r in replay for c in (list(r) + [0] * max_outer)[:max_outer]]
            rkeep = (ctypes.c_int * len(flat))(*flat)
            p.replay_host = ctypes.cast(rkeep, ctypes.POINTER(ctypes.c_int))
        st = (Stats * self.count)()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_batch_solve(self.b, vp, up, ctypes.byref(p), st)
        self._check(rc)
        return us, [s.to_dict() for s in st]

    def info(self):
        bi = BatchInfo()
        self._check(self.lib.tvdeblur_batch_get_info(self.b, ctypes.byref(bi)))
        n = bi.n_candidates
        return {"count": bi.count, "line_threads": bi.line_threads, "tables_in_lds": bool(bi.tables_in_lds),
                "from_cache": bool(bi.from_cache), "candidates": list(bi.cand_threads[:n]),
                "candidate_us": list(bi.cand_us[:n]), "gemm_us": bi.gemm_us, "gemm64_us": bi.gemm64_us,
                "gemm_tile": bi.gemm_tile,
                "transform": {1: "fft", 2: "gemm"}.get(bi.transform, "none"),
                "graph_launches": int(bi.graph_launches),
                "time_setup_s": bi.time_setup_s, "time_inner_s": bi.time_inner_s}


class AlphaSweep:
    """Restorations of one image for many regularisation parameters alpha in
    one batched solve: the batching form with one slot per alpha, all slots
    reading the same observed image (the batch never writes v).  This is the
    alpha study behind the paper's restoration-error comparison of the
    boundary conditions (Section 5: the best alpha and the error it reaches
    under each BC); each restoration is the single-image solve of eq. (fp)
    with that alpha."""

    def __init__(self, shape, psf, bc, alphas, precision="f32_mixed", stream=None):
        alphas = [float(a) for a in alphas]
        if not alphas or not all(a > 0.0 and np.isfinite(a) for a in alphas):
            raise ValueError("alphas must be a non-empty list of positive finite values")
        self.alphas = alphas
        self.shape = (int(shape[0]), int(shape[1]))
        self.batch = TVDeblurBatch([self.shape] * len(alphas), [psf] * len(alphas), bc, precision, stream)

    def solve(self, v, beta=0.05, max_outer=10, inner_tol=1e-6, max_inner=100, precond="x_d", fp_tol=0.0,
              use_graph=True, outs=None, replay=None, transform="auto"):
        """Returns (restorations, per-alpha stats), in the order of alphas."""
        return self.batch.solve([v] * len(self.alphas), self.alphas, beta=beta, max_outer=max_outer,
                                inner_tol=inner_tol, max_inner=max_inner, precond=precond, fp_tol=fp_tol,
                                use_graph=use_graph, outs=outs, replay=replay, transform=transform)

    def info(self):
        return self.batch.info()

    def close(self):
        self.batch.close()


class TVDeblurSignals:
    """Many independent 1D signals (tvdeblur_signals_*): each its own length,
    PSF and BC; every solve is one kernel launch.  Signals travel packed back
    to back in one float64 device tensor (offsets() gives where each starts)."""

    def __init__(self, ns, psfs, bcs, stream=None, reblur=None):
        """reblur: None, or per signal whether to build the reblurring
        system's tables (anti-reflective signals only)."""
        import torch
        self.lib = load()
        self.ns = [int(n) for n in ns]
        self.count = len(self.ns)
        if len(psfs) != self.count or len(bcs) != self.count:
            raise ValueError("one PSF and one BC per signal")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = stream.device
        self._psfs = [np.ascontiguousarray(np.ravel(h), dtype=np.float64) for h in psfs]
        descs = (SignalDesc * self.count)()
        rb = [False] * self.count if reblur is None else list(reblur)
        if len(rb) != self.count:
            raise ValueError("one reblur flag per signal")
        for i, (n, h, bc) in enumerate(zip(self.ns, self._psfs, bcs)):
            descs[i].n, descs[i].plen, descs[i].bc, descs[i].reblur = n, h.size, BC[bc], 1 if rb[i] else 0
            descs[i].psf_host = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_signals_create(ctypes.byref(s), self.count, descs,
                                                  ctypes.c_void_p(stream.cuda_stream))
        if rc != TVD_OK:
            raise TvdError(rc, self.lib.tvdeblur_signals_last_error(None).decode())
        self.s = s
        self.total = sum(self.ns)

    def offsets(self):
        return [int(x) for x in np.concatenate([[0], np.cumsum(self.ns)[:-1]])]

    def pack(self, signals):
        """Device tensor holding the given 1D arrays back to back."""
        import torch
        flat = np.concatenate([np.ravel(np.asarray(x, dtype=np.float64)) for x in signals])
        if flat.size != self.total:
            raise ValueError(f"signals hold {flat.size} samples, the batch {self.total}")
        return torch.tensor(flat, dtype=torch.float64, device=self.device)

    def unpack(self, t):
        a = t.detach().cpu().numpy()
        return [a[o:o + n].copy() for o, n in zip(self.offsets(), self.ns)]

    def close(self):
        if getattr(self, "s", None):
            self.lib.tvdeblur_signals_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, v, alphas, beta=0.1, betas=None, precond="x_d", max_outer=100, fp_tol=1e-3, inner_tol=1e-6,
              max_inner=1000, replay=None, out=None, system="normal", allow_breakdown=False):
        """v: packed float64 device tensor.  precond: one name for all or a
        list per signal (for the reblurring system 'none', 'diag', 'p',
        'd_p', 'p_d').  system: 'normal' (eq. (fp), PCG) or 'reblur' (eq.
        (fpp), PBiCGstab), one for all or a list.  replay: None or per signal
        max_outer counts.  allow_breakdown: return normally when a signal
        broke down (its stats say so) instead of raising.  Returns (packed
        restored tensor, list of per-signal stats dicts)."""
        import torch
        for name, t in (("v", v), ("out", out)):
            if t is not None and (t.dtype != torch.float64 or t.numel() != self.total or not t.is_contiguous()
                                  or t.device != self.device):
                raise ValueError(f"{name} must be a contiguous float64 tensor of {self.total} samples on {self.device}")
        if len(alphas) != self.count:
            raise ValueError("one alpha per signal")
        u = out if out is not None else torch.empty_like(v)
        p = SignalParams()
        keep = []
        a = (ctypes.c_double * self.count)(*[float(x) for x in alphas])
        keep.append(a)
        p.alpha_host = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        p.beta = float(beta)
        if betas is not None:
            if len(betas) != self.count:
                raise ValueError("one beta per signal")
            b = (ctypes.c_double * self.count)(*[float(x) for x in betas])
            keep.append(b)
            p.beta_host = ctypes.cast(b, ctypes.POINTER(ctypes.c_double))
        systems = [system] * self.count if isinstance(system, str) else list(system)
        precs = [precond] * self.count if isinstance(precond, str) else list(precond)
        if len(systems) != self.count or len(precs) != self.count:
            raise ValueError("one system and one preconditioner per signal")
        codes = [(REBLUR_PRECOND if sy == "reblur" else PRECOND)[pr] for sy, pr in zip(systems, precs)]
        pc = (ctypes.c_int * self.count)(*codes)
        sy = (ctypes.c_int * self.count)(*[{"normal": 0, "reblur": 1}[x] for x in systems])
        keep += [pc, sy]
        p.precond_host = ctypes.cast(pc, ctypes.POINTER(ctypes.c_int))
        p.system_host = ctypes.cast(sy, ctypes.POINTER(ctypes.c_int))
        p.max_outer, p.fp_tol, p.inner_tol, p.max_inner = int(max_outer), float(fp_tol), float(inner_tol), int(max_inner)
        if replay is not None:
            if len(replay) != self.count:
                raise ValueError("one replay row per signal")
            rows = []
            for r in replay:
                if len(r) > int(max_outer):
                    raise ValueError("replay row longer than max_outer")
                rows.append(list(r) + [0] * (int(max_outer) - len(r)))
            rp = (ctypes.c_int * (self.count * int(max_outer)))(*[int(x) for row in rows for x in row])
            keep.append(rp)
            p.replay_host = ctypes.cast(rp, ctypes.POINTER(ctypes.c_int))
        stats = (Stats * self.count)()
        with torch.cuda.device(self.device):
            rc = self.lib.tvdeblur_signals_solve(self.s, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                                 ctypes.byref(p), stats)
        del keep
        if rc != TVD_OK and not (allow_breakdown and ERRORS.get(rc) == "TVD_EBREAKDOWN"):
            raise TvdError(rc, self.lib.tvdeblur_signals_last_error(self.s).decode())
        return u, [s.to_dict() for s in stats]
