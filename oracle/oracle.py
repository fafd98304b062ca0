"""ctypes marshalling for the plain FP64 oracle (oracle.c).  Test infrastructure only.

Arrays follow the shared conventions: scalar fields ``(n3, n2, n1)``, vector
fields SoA ``(d, n3, n2, n1)`` (for d < 3 the trailing axes have length 1),
voxel linear index ``i + n1 (j + n2 k)``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_lib = None

ROUTE_PROJECTED, ROUTE_GREEN, ROUTE_DENSE = 0, 1, 2


class _Prob(C.Structure):
    _fields_ = [("d", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("n_phases", C.c_int),
                ("phase", C.c_void_p), ("C21", C.c_void_p), ("rho", C.c_void_p),
                ("dt", C.c_double), ("beta", C.c_double), ("gamma_nm", C.c_double), ("damp", C.c_void_p),
                ("diff_rule", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("route", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("green_tol", C.c_double), ("replay", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        P = C.POINTER(_Prob)
        L.or_fftn.argtypes = [vp, i, vp, i]
        L.or_xi.argtypes = [i, i, d]
        L.or_xi.restype = d
        L.or_xi_rule.argtypes = [i, i, d, i]
        L.or_xi_rule.restype = d
        for f in ("or_apply", "or_precond", "or_div_stress", "or_stress"):
            getattr(L, f).argtypes = [P, vp, vp]
        L.or_deriv.argtypes = [P, vp, i, vp]
        L.or_reference_medium.argtypes = [P, vp, vp]
        L.or_pcg.argtypes = [P, vp, vp, vp, d, d, i, i, vp]
        L.or_pcg.restype = i
        L.or_lu_factor.argtypes = [vp, i, vp]
        L.or_lu_factor.restype = i
        L.or_lu_solve.argtypes = [vp, i, vp, vp]
        L.or_assemble.argtypes = [P, vp]
        L.or_dense_constrained.argtypes = [P, vp, vp, vp, vp]
        L.or_dense_constrained.restype = i
        L.or_green_matrix.argtypes = [P, vp, i, d, i, vp, vp]
        L.or_green_matrix.restype = i
        L.or_newmark.argtypes = [P, vp, i, C.POINTER(_Opts), i, vp, i, vp, vp, vp, vp, vp, vp, vp]
        L.or_newmark.restype = i
        L.or_explicit.argtypes = [P, vp, i, i, vp, i, vp, vp, vp, vp, vp, vp, vp]
        L.or_explicit.restype = i
        L.or_omega2_max.argtypes = [P, vp, i]
        L.or_omega2_max.restype = d
        L.or_conv3d_fwd.argtypes = [vp, vp, vp, vp, i, i, vp]
        L.or_conv3d_bwd_data.argtypes = [vp, vp, vp, i, i, vp]
        L.or_conv3d_bwd_weight.argtypes = [vp, vp, vp, vp, i, i, vp]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """Holds contiguous copies of the problem arrays and the ctypes struct."""

    def __init__(self, dim: int, n: Sequence[int], L: Sequence[float], phase_id: np.ndarray,
                 C21: np.ndarray, rho: np.ndarray, dt: float, beta: float = 0.25,
                 gamma_nm: float = 0.5, damping=None, diff_rule: int = 0):
        self.dim = int(dim)
        nn = [int(x) for x in n] + [1] * (3 - len(n))
        self.n = tuple(nn)
        self.N = nn[0] * nn[1] * nn[2]
        self.phase = np.ascontiguousarray(phase_id, dtype=np.uint16).reshape(-1)
        assert self.phase.size == self.N
        self.C21 = _f64(C21).reshape(-1, 21)
        self.rho = _f64(rho).reshape(-1)
        self.dt, self.beta, self.gamma_nm = float(dt), float(beta), float(gamma_nm)
        LL = [float(x) for x in L] + [1.0] * (3 - len(L))
        self.damp = None if damping is None else _f64(damping).reshape(-1)
        self.s = _Prob(self.dim, (C.c_int * 3)(*nn), (C.c_double * 3)(*LL), self.C21.shape[0],
                       self.phase.ctypes.data, self.C21.ctypes.data, self.rho.ctypes.data,
                       self.dt, self.beta, self.gamma_nm, None if self.damp is None else self.damp.ctypes.data,
                       int(diff_rule))
        self.diff_rule = int(diff_rule)

    @classmethod
    def from_problem(cls, pb) -> "OracleProblem":
        return cls(pb.dim, pb.n, pb.L, pb.phase_id, pb.C21, pb.rho, pb.dt, pb.beta, pb.gamma_nm,
                   getattr(pb, "damping", None), getattr(pb, "diff_rule", 0))

    @property
    def field_shape(self):
        return (self.dim, self.n[2], self.n[1], self.n[0])

    def _vec(self, u) -> np.ndarray:
        u = _f64(u)
        assert u.size == self.dim * self.N, (u.shape, self.field_shape)
        return u

    # --- operator pieces -------------------------------------------------
    def apply(self, u) -> np.ndarray:
        u = self._vec(u)
        out = np.empty(self.field_shape)
        lib().or_apply(C.byref(self.s), _p(u), _p(out))
        return out

    def precond(self, r) -> np.ndarray:
        r = self._vec(r)
        out = np.empty(self.field_shape)
        lib().or_precond(C.byref(self.s), _p(r), _p(out))
        return out

    def div_stress(self, u) -> np.ndarray:
        u = self._vec(u)
        out = np.empty(self.field_shape)
        lib().or_div_stress(C.byref(self.s), _p(u), _p(out))
        return out

    def stress(self, u) -> np.ndarray:
        u = self._vec(u)
        out = np.empty((self.dim, self.dim) + self.field_shape[1:])
        lib().or_stress(C.byref(self.s), _p(u), _p(out))
        return out

    def deriv(self, f, k: int) -> np.ndarray:
        f = _f64(f)
        out = np.empty(self.field_shape[1:])
        lib().or_deriv(C.byref(self.s), _p(f), int(k), _p(out))
        return out

    def reference_medium(self):
        Cb = np.empty(81)
        rb = np.empty(1)
        lib().or_reference_medium(C.byref(self.s), _p(Cb), _p(rb))
        return Cb.reshape(3, 3, 3, 3), float(rb[0])

    # --- solvers -----------------------------------------------------------
    def mask_of(self, gamma_idx) -> np.ndarray:
        m = np.zeros((self.dim, self.N), dtype=np.uint8)
        m[:, np.asarray(gamma_idx, dtype=np.int64)] = 1
        return m.reshape(self.field_shape)

    def pcg(self, b, x0=None, fixed=None, bref=None, tol=1e-10, max_iter=1000, fixed_iters=-1):
        b = self._vec(b)
        x = np.zeros(self.field_shape) if x0 is None else self._vec(x0).copy()
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        if bref is None:
            bref = float(np.linalg.norm(b))
        rel = np.zeros(1)
        it = lib().or_pcg(C.byref(self.s), _p(b), _p(x), _p(fx), float(bref), float(tol),
                          int(max_iter), int(fixed_iters), _p(rel))
        return x, it, float(rel[0])

    def assemble(self) -> np.ndarray:
        n = self.dim * self.N
        A = np.empty((n, n))
        lib().or_assemble(C.byref(self.s), _p(A))
        return A

    def dense_constrained(self, A, b, fixed, x) -> np.ndarray:
        x = self._vec(x).copy()
        st = lib().or_dense_constrained(C.byref(self.s), _p(_f64(A)), _p(self._vec(b)),
                                        _p(np.ascontiguousarray(fixed, dtype=np.uint8)), _p(x))
        if st != 0:
            raise RuntimeError("singular constrained system")
        return x

    def green_matrix(self, gamma_idx, tol=1e-12, max_iter=2000):
        g = np.ascontiguousarray(gamma_idx, dtype=np.int64)
        nd = self.dim * g.size
        G = np.empty((nd, nd))
        its = np.empty(nd, dtype=np.int32)
        st = lib().or_green_matrix(C.byref(self.s), _p(g), int(g.size), float(tol), int(max_iter),
                                   _p(G), _p(its))
        if st != 0:
            raise RuntimeError("Green-matrix solve did not converge")
        return G, its

    def newmark(self, gamma_idx, U, n_steps, route=ROUTE_PROJECTED, tol=1e-10, max_iter=1000,
                green_tol=1e-12, replay=None, per_point=False, u0=None, v0=None, want_F=False):
        """Run the Newmark loop; returns dict(u=(n_steps, d, ...), iters, F, v, a)."""
        g = np.ascontiguousarray(gamma_idx, dtype=np.int64)
        Uarr = _f64(U).reshape(-1)
        rp = None
        if replay is not None:
            rp = np.ascontiguousarray(replay, dtype=np.int32).reshape(-1)
            assert rp.size == 2 * n_steps
        opts = _Opts(int(route), float(tol), int(max_iter), float(green_tol), _p(rp))
        n = self.dim * self.N
        uh = np.empty((n_steps,) + self.field_shape)
        Fh = np.empty((n_steps, self.dim * g.size)) if want_F else None
        its = np.empty((n_steps, 2), dtype=np.int32)
        v = np.empty(self.field_shape)
        a = np.empty(self.field_shape)
        u0a = None if u0 is None else self._vec(u0)
        v0a = None if v0 is None else self._vec(v0)
        st = lib().or_newmark(C.byref(self.s), _p(g), int(g.size), C.byref(opts), int(n_steps),
                              _p(Uarr), int(bool(per_point)), _p(u0a), _p(v0a), _p(uh), _p(Fh),
                              _p(its), _p(v), _p(a))
        if st != 0:
            raise RuntimeError("oracle Newmark failed with status %d" % st)
        return {"u": uh, "iters": its, "F": Fh, "v": v, "a": a}


    def explicit(self, gamma_idx, Udot, n_steps, per_point=False, u0=None, v0=None, want_v=False, want_F=False):
        """Central-difference run (beta = 0, gamma = 1/2) with the velocity Udot prescribed on
        Gamma; returns dict(u=(n_steps, d, ...), v (history if want_v), F, v_last, a_last)."""
        g = np.ascontiguousarray(gamma_idx, dtype=np.int64)
        Ud = _f64(Udot).reshape(-1)
        uh = np.empty((n_steps,) + self.field_shape)
        vh = np.empty((n_steps,) + self.field_shape) if want_v else None
        Fh = np.empty((n_steps, self.dim * g.size)) if want_F else None
        v = np.empty(self.field_shape)
        a = np.empty(self.field_shape)
        u0a = None if u0 is None else self._vec(u0)
        v0a = None if v0 is None else self._vec(v0)
        st = lib().or_explicit(C.byref(self.s), _p(g), int(g.size), int(n_steps), _p(Ud), int(bool(per_point)),
                               _p(u0a), _p(v0a), _p(uh), _p(vh), _p(Fh), _p(v), _p(a))
        if st != 0:
            raise RuntimeError("oracle explicit run failed")
        return {"u": uh, "v": vh, "F": Fh, "v_last": v, "a_last": a}

    def omega2_max(self, x0, iters):
        """Power-iteration estimate of the largest omega^2 of K x = omega^2 rho x from the start
        vector x0; returns (omega^2, last normalised iterate)."""
        x = self._vec(x0).copy()
        lam = lib().or_omega2_max(C.byref(self.s), _p(x), int(iters))
        return float(lam), x


# --- free functions ------------------------------------------------------------
def fftn(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Own radix-2 transform of a complex array shaped (n3, n2, n1) / (n2, n1) / (n1,)."""
    x = np.ascontiguousarray(a, dtype=np.complex128).copy()
    shp = x.shape[::-1]  # fastest first
    n = (C.c_int * 3)(*(list(shp) + [1] * (3 - len(shp))))
    lib().or_fftn(_p(x), 3, n, int(sign))
    return x


def xi(k: int, n: int, L: float) -> float:
    return float(lib().or_xi(int(k), int(n), float(L)))


def xi_rule(k: int, n: int, L: float, rule: int) -> float:
    """Frequency of bin k under a differentiation rule (0 spectral, 1 and 2 centred differences)."""
    return float(lib().or_xi_rule(int(k), int(n), float(L), int(rule)))


def lu_factor(A: np.ndarray):
    LU = _f64(A).copy()
    n = LU.shape[0]
    piv = np.empty(n, dtype=np.int32)
    if lib().or_lu_factor(_p(LU), n, _p(piv)) != 0:
        raise RuntimeError("zero pivot")
    return LU, piv


def lu_solve(LU, piv, b) -> np.ndarray:
    x = _f64(b).copy()
    lib().or_lu_solve(_p(LU), LU.shape[0], _p(piv), _p(x))
    return x


def conv3d_fwd(x, w, bias, n):
    """x (cin, n3, n2, n1), w (cout, cin, 3, 3, 3), bias (cout,) -> y (cout, n3, n2, n1)."""
    x, w = _f64(x), _f64(w)
    cout, cin = w.shape[0], w.shape[1]
    nn = (C.c_int * 3)(*n)
    y = np.empty((cout,) + x.shape[1:])
    b = None if bias is None else _f64(bias)
    lib().or_conv3d_fwd(_p(x), _p(w), _p(b), _p(y), cin, cout, nn)
    return y


def conv3d_bwd_data(dy, w, n):
    dy, w = _f64(dy), _f64(w)
    cout, cin = w.shape[0], w.shape[1]
    dx = np.empty((cin,) + dy.shape[1:])
    lib().or_conv3d_bwd_data(_p(dy), _p(w), _p(dx), cin, cout, (C.c_int * 3)(*n))
    return dx


def conv3d_bwd_weight(x, dy, cin, cout, n):
    x, dy = _f64(x), _f64(dy)
    dw = np.empty((cout, cin, 3, 3, 3))
    db = np.empty(cout)
    lib().or_conv3d_bwd_weight(_p(x), _p(dy), _p(dw), _p(db), cin, cout, (C.c_int * 3)(*n))
    return dw, db
