"""Python binding of libnewmark.so (the C ABI of include/newmark.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Device buffers are torch tensors (used for device memory only).
The binding refuses to run without the built library; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

# PyTorch bundles a HIP runtime under the same soname as the system one.  Importing
# PyTorch before the library is loaded makes the library bind to that same runtime (one
# device context, shared streams and events); loaded the other way round the process
# would hold two runtimes and PyTorch would find no GPU.
try:
    import torch as _torch  # noqa: F401
except ImportError:
    _torch = None

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnewmark.so")

NM_OK, NM_EINVAL, NM_EUNSUPPORTED, NM_ENOMEM, NM_ENOTCONV, NM_ESINGULAR, NM_ENAN, NM_EHIP = 0, -1, -2, -3, -4, -5, -6, -7
NM_FP64, NM_FP32 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
ROUTE_AUTO, ROUTE_GREEN, ROUTE_PROJECTED = 0, 1, 2
WS_COLD, WS_PREV, WS_TAYLOR, WS_LEARNED = 0, 1, 2, 3
DIFF_SPECTRAL, DIFF_CENTRED2, DIFF_CENTRED4 = 0, 1, 2

EXPORTED = ("nm_newmark_init", "nm_newmark_step", "nm_apply_operator", "nm_precond_apply", "nm_pcg_solve",
            "nm_get_state", "nm_set_state", "nm_state_device_ptrs", "nm_green_matrix", "nm_green_solve",
            "nm_get_stream", "nm_profile_passes",
            "nm_net_create", "nm_net_destroy", "nm_net_num_params", "nm_net_get_params", "nm_net_set_params",
            "nm_net_forward", "nm_net_train_step", "nm_net_gradients", "nm_conv3d_bf16", "nm_conv3d_bf16_noalloc",
            "nm_ws_attach",
            "nm_ws_features", "nm_ws_target", "nm_ws_predict", "nm_ws_residual_sample", "nm_ws_train_residual",
            "nm_explicit_step", "nm_omega2_max", "nm_last_error", "nm_destroy")


class NewmarkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"newmark error {code}: {msg}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("n_phases", C.c_int),
                ("phase_id", C.c_void_p), ("C_voigt", C.c_void_p), ("rho", C.c_void_p),
                ("gamma_idx", C.c_void_p), ("n_gamma", C.c_int64), ("u0", C.c_void_p), ("v0", C.c_void_p),
                ("dt", C.c_double), ("beta", C.c_double), ("gamma_nm", C.c_double), ("damping", C.c_void_p),
                ("diff_rule", C.c_int)]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("route", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("inner_tol", C.c_double), ("max_sweeps", C.c_int), ("warm_start", C.c_int),
                ("green_tol", C.c_double), ("compute_reaction", C.c_int), ("true_residual", C.c_int),
                ("green_in", C.c_void_p), ("green_progress", C.c_void_p), ("green_progress_user", C.c_void_p),
                ("green_batch", C.c_int)]


GREEN_PROGRESS = C.CFUNCTYPE(None, C.c_int64, C.c_int64, C.c_void_p)


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int * 2), ("sweeps", C.c_int), ("inner_iters", C.c_int), ("relres", C.c_double),
                ("relres0", C.c_double), ("t_step_ms", C.c_double), ("t_warm_ms", C.c_double)]

    def as_dict(self):
        return {"iters": list(self.iters), "sweeps": self.sweeps, "inner_iters": self.inner_iters,
                "relres": self.relres, "relres0": self.relres0, "t_step_ms": self.t_step_ms, "t_warm_ms": self.t_warm_ms}


_lib = None


def hip_runtimes_loaded():
    """Paths of the HIP runtime libraries mapped into this process (Linux)."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def load_library():
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libnewmark.so is not built (run __graft_entry__.build() or "
                           "python paper_2211_08263_amd/build.py); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    runtimes = hip_runtimes_loaded()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process (%s); import torch before anything "
                           "that loads the ROCm HIP runtime" % ", ".join(sorted(runtimes)))
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    L.nm_newmark_init.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), vp, C.POINTER(vp)]
    L.nm_newmark_step.argtypes = [vp, vp, i, C.POINTER(StepStats)]
    L.nm_apply_operator.argtypes = [vp, vp, vp, i]
    L.nm_precond_apply.argtypes = [vp, vp, vp, i]
    L.nm_pcg_solve.argtypes = [vp, vp, vp, i, d, i, i, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.nm_get_state.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_int64)]
    L.nm_set_state.argtypes = [vp, vp, vp, vp, C.c_int64]
    L.nm_state_device_ptrs.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
    L.nm_green_matrix.argtypes = [vp, vp]
    L.nm_green_solve.argtypes = [vp, vp, vp]
    L.nm_profile_passes.argtypes = [vp, i, vp, vp, i, i, C.POINTER(C.c_double)]
    L.nm_net_create.argtypes = [C.c_ulonglong, C.POINTER(vp)]
    L.nm_net_destroy.argtypes = [vp]
    L.nm_net_destroy.restype = None
    L.nm_net_num_params.argtypes = [vp]
    L.nm_net_num_params.restype = C.c_long
    L.nm_net_get_params.argtypes = [vp, vp]
    L.nm_net_set_params.argtypes = [vp, vp]
    L.nm_net_forward.argtypes = [vp, vp, vp, vp, vp]
    L.nm_net_train_step.argtypes = [vp, vp, vp, vp, vp, C.c_float, C.POINTER(C.c_float)]
    L.nm_net_gradients.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(C.c_float)]
    L.nm_conv3d_bf16.argtypes = [vp, i, vp, i, i, i, vp, vp, vp, vp, vp, vp, vp]
    L.nm_conv3d_bf16_noalloc.argtypes = [vp, i, vp, i, i, i, vp, vp, vp, vp, vp, vp, vp]
    L.nm_ws_attach.argtypes = [vp, vp]
    L.nm_ws_features.argtypes = [vp, vp]
    L.nm_ws_target.argtypes = [vp, vp]
    L.nm_ws_predict.argtypes = [vp, vp]
    L.nm_ws_residual_sample.argtypes = [vp, vp, C.c_int, vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
    L.nm_ws_train_residual.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_int, C.c_float,
                                       C.POINTER(C.c_float)]
    L.nm_explicit_step.argtypes = [vp, vp, i, i, C.POINTER(StepStats)]
    L.nm_omega2_max.argtypes = [vp, vp, i, C.POINTER(C.c_double)]
    L.nm_get_stream.argtypes = [vp]
    L.nm_get_stream.restype = vp
    L.nm_last_error.argtypes = [vp]
    L.nm_last_error.restype = C.c_char_p
    L.nm_destroy.argtypes = [vp]
    L.nm_destroy.restype = None
    _lib = L
    return L


@dataclass
class Options:
    precision: int = PREC_FP64
    route: int = ROUTE_PROJECTED
    tol: float = 1e-8
    max_iter: int = 1000
    inner_tol: float = 1e-5
    max_sweeps: int = 20
    warm_start: int = WS_PREV
    green_tol: float = 0.0
    compute_reaction: int = 0
    true_residual: int = 0
    green_in: Optional[np.ndarray] = None  # stored Green matrix to reuse (GREEN route)
    green_progress: object = None  # callable(done, total) after each unit-force solve (GREEN route)
    green_batch: int = 0  # unit-force solves run together: 0 automatic, 1 one at a time, k >= 2 k at a time


class Context:
    """An initialised solver (nm_newmark_init); call close() or use as a context manager."""

    def __init__(self, ptr, problem_arrays, dim, n, n_gamma):
        self._ptr = ptr
        self._keep = problem_arrays
        self.dim = dim
        self.n = n
        self.N = n[0] * n[1] * n[2]
        self.n_gamma = n_gamma

    @property
    def handle(self):
        if not self._ptr:
            raise RuntimeError("context is closed")
        return self._ptr

    def last_error(self) -> str:
        return load_library().nm_last_error(self.handle).decode()

    def check(self, code: int):
        if code != NM_OK:
            raise NewmarkError(code, self.last_error())

    def close(self):
        if self._ptr:
            load_library().nm_destroy(self._ptr)
            self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def newmark_init(dim: int, n: Sequence[int], L: Sequence[float], phase_id, C_voigt, rho, gamma_idx, dt: float,
                 beta: float = 0.25, gamma_nm: float = 0.5, u0=None, v0=None, options: Optional[Options] = None,
                 stream=None, damping=None, diff_rule: int = DIFF_SPECTRAL) -> Context:
    """damping: per-phase viscous coefficients c >= 0 (force -c v), or None; diff_rule: the
    derivative's symbol (DIFF_SPECTRAL, DIFF_CENTRED2, DIFF_CENTRED4)."""
    lib = load_library()
    nn = [int(x) for x in n] + [1] * (3 - len(n))
    LL = [float(x) for x in L] + [1.0] * (3 - len(L))
    ph = np.ascontiguousarray(phase_id, dtype=np.uint16).reshape(-1)
    Cv = _c64(C_voigt).reshape(-1)
    rh = _c64(rho).reshape(-1)
    g = np.ascontiguousarray(gamma_idx, dtype=np.int64).reshape(-1)
    u0a = None if u0 is None else _c64(u0).reshape(-1)
    v0a = None if v0 is None else _c64(v0).reshape(-1)
    dm = None if damping is None else _c64(damping).reshape(-1)
    if dm is not None and dm.size != rh.size:
        raise ValueError("damping needs one coefficient per phase")
    pb = _Problem(int(dim), (C.c_int * 3)(*nn), (C.c_double * 3)(*LL), rh.size, ph.ctypes.data, Cv.ctypes.data,
                  rh.ctypes.data, g.ctypes.data if g.size else None, g.size,
                  None if u0a is None else u0a.ctypes.data, None if v0a is None else v0a.ctypes.data,
                  float(dt), float(beta), float(gamma_nm), None if dm is None else dm.ctypes.data,
                  int(diff_rule))
    o = options or Options()
    gin = None if o.green_in is None else _c64(o.green_in).reshape(-1)
    cb = None
    if o.green_progress is not None:
        user_cb = o.green_progress
        cb = GREEN_PROGRESS(lambda done, total, _u: user_cb(int(done), int(total)))
    op = _Options(o.precision, o.route, o.tol, o.max_iter, o.inner_tol, o.max_sweeps, o.warm_start, o.green_tol,
                  o.compute_reaction, o.true_residual, None if gin is None else gin.ctypes.data,
                  None if cb is None else C.cast(cb, C.c_void_p).value, None, int(o.green_batch))
    out = C.c_void_p()
    code = lib.nm_newmark_init(C.byref(pb), C.byref(op), stream, C.byref(out))
    ctx = Context(out.value, (ph, Cv, rh, g, dm), int(dim), tuple(nn), int(g.size))
    if code != NM_OK:
        msg = ctx.last_error() if out.value else ""
        ctx.close()
        raise NewmarkError(code, msg)
    return ctx


def newmark_init_problem(pb, options: Optional[Options] = None, u0=None, v0=None, stream=None) -> Context:
    """newmark_init from a workloads.Problem."""
    return newmark_init(pb.dim, pb.n, pb.L, pb.phase_id, pb.C21, pb.rho, pb.gamma_idx, pb.dt, pb.beta, pb.gamma_nm,
                        u0=u0, v0=v0, options=options, stream=stream, damping=getattr(pb, "damping", None),
                        diff_rule=getattr(pb, "diff_rule", DIFF_SPECTRAL))


def newmark_step(ctx: Context, U, per_point: bool = False) -> dict:
    Ua = _c64(U).reshape(-1)
    st = StepStats()
    ctx.check(load_library().nm_newmark_step(ctx.handle, Ua.ctypes.data, int(bool(per_point)), C.byref(st)))
    return st.as_dict()


def explicit_step(ctx: Context, Udot, per_point: bool = False, n_steps: int = 1) -> dict:
    """n_steps central-difference steps; Udot holds n_steps rows of prescribed velocities."""
    Ua = _c64(Udot).reshape(-1)
    st = StepStats()
    ctx.check(load_library().nm_explicit_step(ctx.handle, Ua.ctypes.data if Ua.size else None, int(bool(per_point)),
                                              int(n_steps), C.byref(st)))
    return st.as_dict()


def omega2_max(ctx: Context, x, iters: int) -> float:
    """Power-iteration estimate of omega_max^2 (x: device float64 tensor of 3 x N, overwritten)."""
    _check_field(ctx, x)
    import torch
    if x.dtype != torch.float64:
        raise TypeError("float64 start vector expected")
    w = C.c_double(0)
    ctx.check(load_library().nm_omega2_max(ctx.handle, x.data_ptr(), int(iters), C.byref(w)))
    return w.value


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return NM_FP64
    if t.dtype == torch.float32:
        return NM_FP32
    raise TypeError("float64 or float32 tensors expected")


def _check_field(ctx, t):
    if not t.is_cuda or not t.is_contiguous() or t.numel() != 3 * ctx.N:
        raise ValueError("expected a contiguous device tensor of 3 x N values")


def apply_operator(ctx: Context, u, out) -> None:
    """out = A(u) on device tensors (3 x N, float64 or float32); asynchronous on the context stream."""
    _check_field(ctx, u)
    _check_field(ctx, out)
    if u.dtype != out.dtype:
        raise TypeError("u and out must share a dtype")
    ctx.check(load_library().nm_apply_operator(ctx.handle, u.data_ptr(), out.data_ptr(), _dtype_code(u)))


def precond_apply(ctx: Context, r, z) -> None:
    _check_field(ctx, r)
    _check_field(ctx, z)
    if r.dtype != z.dtype:
        raise TypeError("r and z must share a dtype")
    ctx.check(load_library().nm_precond_apply(ctx.handle, r.data_ptr(), z.data_ptr(), _dtype_code(r)))


def pcg_solve(ctx: Context, b, x, masked: bool = False, tol: float = 1e-10, max_iter: int = 1000,
              fixed_iters: int = -1):
    _check_field(ctx, b)
    _check_field(ctx, x)
    it = C.c_int(0)
    rel = C.c_double(0)
    ctx.check(load_library().nm_pcg_solve(ctx.handle, b.data_ptr(), x.data_ptr(), int(bool(masked)), float(tol),
                                          int(max_iter), int(fixed_iters), C.byref(it), C.byref(rel)))
    return it.value, rel.value


def get_state(ctx: Context):
    N, d = ctx.N, ctx.dim
    u = np.empty(d * N)
    v = np.empty(d * N)
    a = np.empty(d * N)
    F = np.empty(max(1, d * ctx.n_gamma))
    step = C.c_int64(0)
    ctx.check(load_library().nm_get_state(ctx.handle, u.ctypes.data, v.ctypes.data, a.ctypes.data, F.ctypes.data,
                                          C.byref(step)))
    shp = (d, ctx.n[2], ctx.n[1], ctx.n[0])
    return {"u": u.reshape(shp), "v": v.reshape(shp), "a": a.reshape(shp), "F": F[: d * ctx.n_gamma],
            "step": step.value}


def set_state(ctx: Context, u, v, a, step: int) -> None:
    ua, va, aa = _c64(u).reshape(-1), _c64(v).reshape(-1), _c64(a).reshape(-1)
    ctx.check(load_library().nm_set_state(ctx.handle, ua.ctypes.data, va.ctypes.data, aa.ctypes.data, int(step)))


def state_device_ptrs(ctx: Context):
    u, v, a = C.c_void_p(), C.c_void_p(), C.c_void_p()
    ctx.check(load_library().nm_state_device_ptrs(ctx.handle, C.byref(u), C.byref(v), C.byref(a)))
    return u.value, v.value, a.value


def green_matrix(ctx: Context) -> np.ndarray:
    nd = ctx.dim * ctx.n_gamma
    G = np.empty((nd, nd))
    ctx.check(load_library().nm_green_matrix(ctx.handle, G.ctypes.data))
    return G


def green_solve(ctx: Context, V) -> np.ndarray:
    """G^-1 V with the context's device LU factors (GREEN route)."""
    Va = _c64(V).reshape(-1)
    X = np.empty_like(Va)
    ctx.check(load_library().nm_green_solve(ctx.handle, Va.ctypes.data, X.ctypes.data))
    return X


OPERATOR_PASSES = ("x_fwd", "y_deriv", "z_strain", "x_stress", "y_div", "z_div", "x_inv_inertia")
PRECOND_PASSES = ("x_fwd", "y_fwd3", "z_precond", "y_inv3", "x_inv")


def profile_passes(ctx: Context, which: int, u, out, reps: int = 10):
    """Average event-timed duration (ms) of every pass of one operator (0) or preconditioner (1) apply."""
    _check_field(ctx, u)
    _check_field(ctx, out)
    ms = (C.c_double * 9)()
    ctx.check(load_library().nm_profile_passes(ctx.handle, int(which), u.data_ptr(), out.data_ptr(),
                                               _dtype_code(u), int(reps), ms))
    names = OPERATOR_PASSES if which == 0 else PRECOND_PASSES
    return {nm: ms[i] for i, nm in enumerate(names)}


def get_stream(ctx: Context) -> int:
    return load_library().nm_get_stream(ctx.handle) or 0


# --------------------------------------------------------------------------------------------
# Learned warm start
# --------------------------------------------------------------------------------------------
def _grid(n):
    return (C.c_int * 3)(*[int(x) for x in n])


def _stream_arg(stream):
    return None if stream is None else C.c_void_p(int(stream))


class Net:
    """The warm-start network (nm_net_*).  Device buffers are torch tensors."""

    def __init__(self, seed: int = 0):
        lib = load_library()
        out = C.c_void_p()
        code = lib.nm_net_create(int(seed), C.byref(out))
        if code != NM_OK:
            raise NewmarkError(code, "nm_net_create failed")
        self._ptr = out.value

    @property
    def handle(self):
        if not self._ptr:
            raise RuntimeError("network is closed")
        return self._ptr

    def close(self):
        if self._ptr:
            load_library().nm_net_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self) -> int:
        return int(load_library().nm_net_num_params(self.handle))

    def get_params(self) -> np.ndarray:
        w = np.empty(self.num_params(), dtype=np.float32)
        _chk(load_library().nm_net_get_params(self.handle, w.ctypes.data), "get_params")
        return w

    def set_params(self, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.num_params()
        _chk(load_library().nm_net_set_params(self.handle, w.ctypes.data), "set_params")

    def forward(self, grid, feat, pred, stream=None) -> None:
        _chk(load_library().nm_net_forward(self.handle, _stream_arg(stream), _grid(grid), feat.data_ptr(),
                                           pred.data_ptr()), "forward")

    def train_step(self, grid, feat, target, lr: float, stream=None) -> float:
        loss = C.c_float(0)
        _chk(load_library().nm_net_train_step(self.handle, _stream_arg(stream), _grid(grid), feat.data_ptr(),
                                              target.data_ptr(), float(lr), C.byref(loss)), "train_step")
        return float(loss.value)

    def gradients(self, grid, feat, target, stream=None):
        g = np.empty(self.num_params(), dtype=np.float32)
        loss = C.c_float(0)
        _chk(load_library().nm_net_gradients(self.handle, _stream_arg(stream), _grid(grid), feat.data_ptr(),
                                             target.data_ptr(), g.ctypes.data, C.byref(loss)), "gradients")
        return g, float(loss.value)


def _chk(code, what):
    if code != NM_OK:
        raise NewmarkError(code, what)


def conv3d_bf16(mode, grid, cinp, cin, cout, x=None, w=None, bias=None, dy=None, out=None, stream=None,
                noalloc=False):
    """One network layer's kernel on caller buffers (see nm_conv3d_bf16; noalloc selects
    nm_conv3d_bf16_noalloc, which allocates no device memory)."""
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    ba = None if bias is None else np.ascontiguousarray(bias, dtype=np.float32)
    dw = np.zeros((cout, cin, 27), dtype=np.float32)
    db = np.zeros(cout, dtype=np.float32)
    fn = load_library().nm_conv3d_bf16_noalloc if noalloc else load_library().nm_conv3d_bf16
    _chk(fn(_stream_arg(stream), int(mode), _grid(grid), int(cinp), int(cin), int(cout),
                                       None if x is None else x.data_ptr(), None if wa is None else wa.ctypes.data,
                                       None if ba is None else ba.ctypes.data, None if dy is None else dy.data_ptr(),
                                       None if out is None else out.data_ptr(), dw.ctypes.data, db.ctypes.data),
         "conv3d_bf16")
    return dw, db


def ws_attach(ctx: Context, net) -> None:
    ctx.check(load_library().nm_ws_attach(ctx.handle, None if net is None else net.handle))
    ctx._net = net


def ws_features(ctx: Context, feat=None) -> None:
    ctx.check(load_library().nm_ws_features(ctx.handle, None if feat is None else feat.data_ptr()))


def ws_predict(ctx: Context, x0) -> None:
    ctx.check(load_library().nm_ws_predict(ctx.handle, x0.data_ptr()))


def ws_target(ctx: Context, target) -> None:
    ctx.check(load_library().nm_ws_target(ctx.handle, target.data_ptr()))


def ws_residual_sample(ctx: Context, U_next, feat, rp, per_point: bool = False):
    """Features and projected residual of the predictor for the coming step; returns
    (s, cref, crefM)."""
    U = _c64(U_next).reshape(-1)
    sv, cv, cm = C.c_double(), C.c_double(), C.c_double()
    ctx.check(load_library().nm_ws_residual_sample(ctx.handle, U.ctypes.data, int(bool(per_point)), feat.data_ptr(),
                                                   rp.data_ptr(), C.byref(sv), C.byref(cv), C.byref(cm)))
    return sv.value, cv.value, cm.value


def ws_train_residual(ctx: Context, feat, rp, s: float, cref: float, lr: float, metric: int = 0) -> float:
    loss = C.c_float()
    ctx.check(load_library().nm_ws_train_residual(ctx.handle, feat.data_ptr(), rp.data_ptr(), float(s), float(cref),
                                                  int(metric), float(lr), C.byref(loss)))
    return loss.value
