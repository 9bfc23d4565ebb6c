"""ctypes binding of the plain-C FP64 oracle (``mgseg_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgseg_oracle.c")
_LIB = os.path.join(_HERE, "libmgseg_oracle.so")

FIELDS = {"z": 0, "d": 1, "w": 2, "fit": 3, "phi": 4, "F": 5, "A": 6, "B": 7, "C": 8,
          "D": 9, "S": 10, "f": 11, "g": 12, "lo": 13, "hi": 14, "phic": 15}


# -O3 without -march=native: the library may be built on another host than the
# one that runs it; no fast-math (the oracle's arithmetic is plain IEEE FP64)
OPT_FLAGS = ("-O3",)


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with the host compiler (-O3, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *OPT_FLAGS, "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("model", C.c_int), ("mu", C.c_double), ("lambda1", C.c_double),
                ("lambda2", C.c_double), ("theta", C.c_double), ("nu", C.c_double),
                ("eps", C.c_double), ("eps_tv_px", C.c_double), ("beta", C.c_double),
                ("sigma_g", C.c_double), ("sigma_d", C.c_double), ("Sigma", C.c_double),
                ("M", C.c_double), ("nu1", C.c_int), ("nu2", C.c_int), ("levels", C.c_int),
                ("coarse_iters", C.c_int), ("coarse_rtol", C.c_double), ("order", C.c_int), ("smoother", C.c_int),
                ("obstacle", C.c_int), ("scaled", C.c_int), ("run_max", C.c_int)]


@dataclass
class OracleParams:
    model: int = 0            # 0 Spencer-Chen, 1 Rada-Chen
    mu: float = 0.5
    lambda1: float = 6.5025
    lambda2: float = 6.5025
    theta: float = 4.0
    nu: float = 1.0
    eps: float = 1.0
    eps_tv_px: float = 1.0
    beta: float = 16384.0
    sigma_g: float = 1.0
    sigma_d: float = 0.1
    Sigma: float = 2.0
    M: float = 4.0
    nu1: int = 2
    nu2: int = 2
    levels: int = 1
    coarse_iters: int = 10
    coarse_rtol: float = 1e-4  # coarsest solve stops when an iteration moves nothing by more than this share
    order: int = 1            # 0 paper lexicographic lines, 1 four-class line order
    smoother: int = 0         # 0 Hybrid Smoother 2, 1 GSLEX-I, 2 Hybrid Smoother 1, 3 GSLINE-I, 4 NEWT-I,
                              # 5 GSLEX-II, 6 GSLINE-II, 7 NEWT-II
    obstacle: int = 1         # 1 coarse corrections bounded by the fine slack
    scaled: int = 1           # 1 each row divided by delta_eps(psi_ij) > 0
    run_max: int = 0          # 0 maximal runs (Sec. 4.3), else runs cut into near-equal pieces of at most run_max

    def to_c(self) -> _Params:
        p = _Params()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build_oracle())
        dp = C.POINTER(C.c_double)
        _lib.or_create.restype = C.c_void_p
        _lib.or_create.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int, C.POINTER(_Params)]
        _lib.or_destroy.argtypes = [C.c_void_p]
        _lib.or_vcycle.restype = C.c_double
        _lib.or_vcycle.argtypes = [C.c_void_p, dp]
        _lib.or_solve.restype = C.c_int
        _lib.or_solve.argtypes = [C.c_void_p, C.c_double, C.c_int, dp]
        _lib.or_res_norm.restype = C.c_double
        _lib.or_res_norm.argtypes = [C.c_void_p]
        _lib.or_res_norm_rows.restype = C.c_double
        _lib.or_res_norm_rows.argtypes = [C.c_void_p]
        _lib.or_rel_rows.restype = C.c_double
        _lib.or_rel_rows.argtypes = [C.c_void_p]
        _lib.or_set_res0_rows.argtypes = [C.c_void_p, C.c_double]
        _lib.or_energy.restype = C.c_double
        _lib.or_energy.argtypes = [C.c_void_p]
        _lib.or_timemarch.restype = C.c_double
        _lib.or_timemarch.argtypes = [C.c_void_p, C.c_long, C.c_double, C.c_int, C.c_double]
        _lib.or_aos_step.restype = C.c_double
        _lib.or_aos_step.argtypes = [C.c_void_p, C.c_double]
        _lib.or_aos.restype = C.c_int
        _lib.or_aos.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, dp]
        _lib.or_newton_qprime.restype = None
        _lib.or_newton_qprime.argtypes = [C.c_void_p, C.c_int, dp]
        _lib.or_tridiag_solve.restype = None
        _lib.or_tridiag_solve.argtypes = [C.c_int, dp, dp, dp, dp]
        _lib.or_levels.restype = C.c_int
        _lib.or_levels.argtypes = [C.c_void_p]
        _lib.or_level_shape.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        _lib.or_scalars.argtypes = [C.c_void_p, dp]
        _lib.or_set_c.argtypes = [C.c_void_p, C.c_double, C.c_double]
        _lib.or_set_res0.argtypes = [C.c_void_p, C.c_double]
        _lib.or_get.restype = C.c_int
        _lib.or_get.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        _lib.or_set.restype = C.c_int
        _lib.or_set.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        _lib.or_get_labels.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint8)]
        _lib.or_set_labels.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint8)]
        for name in ("or_step_freeze", "or_step_coarsest", "or_step_vcycle_level", "or_step_to_coarse"):
            getattr(_lib, name).argtypes = [C.c_void_p, C.c_int]
        _lib.or_step_sweep.argtypes = [C.c_void_p, C.c_int, C.c_int]
        _lib.or_step_smooth.argtypes = [C.c_void_p, C.c_int, C.c_int]
        _lib.or_step_residual.argtypes = [C.c_void_p, C.c_int, dp, C.c_int]
        _lib.or_step_operator.argtypes = [C.c_void_p, C.c_int, dp]
        _lib.or_step_update_c.argtypes = [C.c_void_p]
        _lib.or_step_area_term.restype = C.c_double
        _lib.or_step_area_term.argtypes = [C.c_void_p, C.c_int]
        _lib.or_restrict.argtypes = [dp, C.c_int, C.c_int, dp]
        _lib.or_prolong.argtypes = [dp, C.c_int, C.c_int, dp]
        _lib.or_hull.restype = C.c_int
        _lib.or_hull.argtypes = [dp, C.c_int, dp]
        _lib.or_box_dense.restype = C.c_int
        _lib.or_box_dense.argtypes = [C.c_int, dp, dp, dp, dp, dp]
        _lib.or_box_tridiag.restype = C.c_int
        _lib.or_box_tridiag.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp]
        _lib.or_line_units.argtypes = [C.POINTER(C.c_uint8), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
        _lib.or_visit_order.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_long)]
        _lib.or_setup_maps.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int, C.POINTER(_Params),
                                       dp, dp, dp, dp, dp]
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def restrict(fine: np.ndarray) -> np.ndarray:
    fine = np.ascontiguousarray(fine, np.float64)
    n, m = fine.shape
    out = np.zeros((n // 2, m // 2))
    _load().or_restrict(_dp(fine), n, m, _dp(out))
    return out


def prolong(coarse: np.ndarray) -> np.ndarray:
    coarse = np.ascontiguousarray(coarse, np.float64)
    nc, mc = coarse.shape
    out = np.zeros((2 * nc, 2 * mc))
    _load().or_prolong(_dp(coarse), nc, mc, _dp(out))
    return out


def hull(points: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(points, np.float64)
    out = np.zeros(2 * 130)
    k = _load().or_hull(_dp(pts), len(pts), _dp(out))
    return out[: 2 * k].reshape(k, 2)


def box_tridiag(lo, di, up, rh, bl, bh):
    """Box-constrained tridiagonal solve of one run (None on a zero pivot)."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (lo, di, up, rh, bl, bh)]
    x = np.zeros(len(di))
    ok = _load().or_box_tridiag(len(di), *[_dp(a) for a in arrs], _dp(x))
    return x if ok else None


def box_dense(M, b, bl, bh):
    """Box-constrained solve of a small dense system (None on a zero pivot)."""
    M = np.ascontiguousarray(M, np.float64)
    arrs = [np.ascontiguousarray(a, np.float64) for a in (b, bl, bh)]
    x = np.zeros(len(b))
    ok = _load().or_box_dense(len(b), _dp(M), *[_dp(a) for a in arrs], _dp(x))
    return x if ok else None


def tridiag_solve(lo, di, up, rhs):
    """The oracle's Thomas solve of lo_k x_{k-1} + di_k x_k + up_k x_{k+1} = rhs_k."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (lo, di, up)]
    x = np.array(rhs, np.float64)
    _load().or_tridiag_solve(len(x), *[_dp(a) for a in arrs], _dp(x))
    return x


def line_units(labels_line, bit, run_max=0):
    """Start position of the unit of every position of a line (visit order);
    run_max 0: maximal runs, else runs cut into pieces of at most run_max."""
    a = np.ascontiguousarray(labels_line, np.uint8)
    out = np.zeros(len(a), np.int32)
    _load().or_line_units(a.ctypes.data_as(C.POINTER(C.c_uint8)), len(a), bit, run_max,
                          out.ctypes.data_as(C.POINTER(C.c_int)))
    return out


def visit_order(s, n, m, order=0):
    """Flat pixel indices in the order sweep s visits an n x m grid."""
    out = np.zeros(n * m, np.int64)
    _load().or_visit_order(s, n, m, order, out.ctypes.data_as(C.POINTER(C.c_long)))
    return out


def setup_maps(image, markers, params: OracleParams):
    z = np.ascontiguousarray(image, np.float64)
    mk = np.ascontiguousarray(markers, np.float64)
    n, m = z.shape
    g, d, w, phi0 = (np.zeros((n, m)) for _ in range(4))
    A1 = np.zeros(1)
    p = params.to_c()
    _load().or_setup_maps(_dp(z), n, m, _dp(mk), len(mk), C.byref(p), _dp(g), _dp(d), _dp(w),
                          _dp(phi0), _dp(A1))
    return dict(g=g, d=d, w=w, phi0=phi0, A1=float(A1[0]))


class Oracle:
    """One image: level hierarchy, FAS V-cycles, single steps, diagnostics."""

    def __init__(self, image, markers, params: OracleParams):
        self.lib = _load()
        z = np.ascontiguousarray(image, np.float64)
        mk = np.ascontiguousarray(markers, np.float64)
        self.params = params
        self._p = params.to_c()
        self.ctx = self.lib.or_create(_dp(z), z.shape[0], z.shape[1], _dp(mk), len(mk),
                                      C.byref(self._p))
        if not self.ctx:
            raise ValueError("oracle: invalid shape / level count")

    def __del__(self):
        if getattr(self, "ctx", None):
            self.lib.or_destroy(self.ctx)
            self.ctx = None

    @property
    def levels(self) -> int:
        return self.lib.or_levels(self.ctx)

    def shape(self, l: int):
        n, m, h = C.c_int(), C.c_int(), C.c_double()
        self.lib.or_level_shape(self.ctx, l, C.byref(n), C.byref(m), C.byref(h))
        return n.value, m.value, h.value

    def scalars(self):
        out = np.zeros(5)
        self.lib.or_scalars(self.ctx, _dp(out))
        return dict(c1=out[0], c2=out[1], A1=out[2], res0=out[3], h0=out[4])

    def get(self, name: str, l: int = 0) -> np.ndarray:
        n, m, _ = self.shape(l)
        out = np.zeros((n, m))
        if self.lib.or_get(self.ctx, l, FIELDS[name], _dp(out)) != 0:
            raise KeyError(name)
        return out

    def set(self, name: str, arr, l: int = 0):
        n, m, _ = self.shape(l)
        a = np.ascontiguousarray(arr, np.float64).reshape(n, m)
        if self.lib.or_set(self.ctx, l, FIELDS[name], _dp(a)) != 0:
            raise KeyError(name)

    def labels(self, l: int = 0) -> np.ndarray:
        n, m, _ = self.shape(l)
        out = np.zeros((n, m), np.uint8)
        self.lib.or_get_labels(self.ctx, l, out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out

    def set_labels(self, lab, l: int = 0):
        a = np.ascontiguousarray(lab, np.uint8)
        self.lib.or_set_labels(self.ctx, l, a.ctypes.data_as(C.POINTER(C.c_uint8)))

    def set_c(self, c1: float, c2: float):
        self.lib.or_set_c(self.ctx, c1, c2)

    def set_res0(self, r0: float):
        self.lib.or_set_res0(self.ctx, r0)

    # --- whole-method entry points
    def vcycle(self):
        eta = C.c_double()
        rel = self.lib.or_vcycle(self.ctx, C.byref(eta))
        return rel, eta.value

    def solve(self, tol=1e-6, max_cycles=50):
        hist = np.zeros(max_cycles)
        k = self.lib.or_solve(self.ctx, tol, max_cycles, _dp(hist))
        return k, hist[: abs(k)]

    def res_norm(self) -> float:
        """Projected residual norm of the paper's rows (eq. abcdrc, each with its delta factor)."""
        return self.lib.or_res_norm(self.ctx)

    def res_norm_rows(self) -> float:
        """Projected residual norm of the rows the smoother holds (divided by delta if scaled)."""
        return self.lib.or_res_norm_rows(self.ctx)

    def rel_rows(self) -> float:
        """The last cycle's relative residual of the smoother's rows."""
        return self.lib.or_rel_rows(self.ctx)

    def set_res0_rows(self, r0: float):
        self.lib.or_set_res0_rows(self.ctx, r0)

    def energy(self) -> float:
        return self.lib.or_energy(self.ctx)

    def timemarch(self, steps, cfl=0.2, crefresh=100, tol=0.0) -> float:
        return self.lib.or_timemarch(self.ctx, steps, cfl, crefresh, tol)

    def aos_step(self, tau: float) -> float:
        """One AOS step of the finest grid (time step tau in units of h/mu), then
        the region means refreshed; returns the relative change of phi."""
        return self.lib.or_aos_step(self.ctx, tau)

    def aos(self, tau: float, eta_tol: float = 1e-4, max_iters: int = 200):
        """AOS steps until the relative change falls below eta_tol: (steps, changes);
        steps is negative when the tolerance was not reached."""
        hist = np.zeros(max_iters)
        k = self.lib.or_aos(self.ctx, tau, eta_tol, max_iters, _dp(hist))
        return k, hist[: abs(k)]

    # --- single steps
    def freeze(self, l=0):
        self.lib.or_step_freeze(self.ctx, l)

    def sweep(self, s, l=0):
        self.lib.or_step_sweep(self.ctx, l, s)

    def smooth(self, iters, l=0):
        self.lib.or_step_smooth(self.ctx, l, iters)

    def coarsest(self, l):
        self.lib.or_step_coarsest(self.ctx, l)

    def vcycle_level(self, l):
        self.lib.or_step_vcycle_level(self.ctx, l)

    def to_coarse(self, l):
        """The coarse problem of level l + 1 from level l's state (restriction, bounds, FAS right-hand side)."""
        self.lib.or_step_to_coarse(self.ctx, l)

    def residual(self, l=0, project=True) -> np.ndarray:
        n, m, _ = self.shape(l)
        out = np.zeros((n, m))
        self.lib.or_step_residual(self.ctx, l, _dp(out), int(project))
        return out

    def operator(self, l=0) -> np.ndarray:
        n, m, _ = self.shape(l)
        out = np.zeros((n, m))
        self.lib.or_step_operator(self.ctx, l, _dp(out))
        return out

    def newton_qprime(self, l=0) -> np.ndarray:
        """NEWT's diagonal term Q' of every cell at the current phi (Sec. 3.2, eq. newtrc)."""
        n, m, _ = self.shape(l)
        out = np.zeros((n, m))
        self.lib.or_newton_qprime(self.ctx, l, _dp(out))
        return out

    def update_c(self):
        self.lib.or_step_update_c(self.ctx)

    def area_term(self, l=0) -> float:
        return self.lib.or_step_area_term(self.ctx, l)
