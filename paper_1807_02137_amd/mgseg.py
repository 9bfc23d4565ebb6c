"""Python binding of libmgseg (argument marshalling only).

Every step of the solver runs in the library's HIP kernels; PyTorch supplies
device memory and the stream.  The binding fails loudly when the built
library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np
import torch

from . import build as _build

FIELD = {"z": 0, "d": 1, "w": 2, "fit": 3, "phi": 4, "F": 5, "lo": 6, "hi": 7, "g": 8, "phi64": 9,
         "labels": 10, "r": 11}
OP = {"freeze": 0, "sweep_A": 1, "sweep_B": 2, "sweep_C": 3, "sweep_D": 4, "smooth": 5, "coarsest": 6,
      "vcycle_from": 7, "residual": 8, "update_c": 9}

STATUS = {0: "ok", 1: "invalid argument", 2: "shape", 3: "out of device memory", 4: "HIP error",
          5: "non-finite residual", 6: "not converged", 7: "invalid state",
          8: "image too large for the no-allocation scratch"}


class MgsegError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("model", C.c_int32), ("mu", C.c_double),
                ("lambda1", C.c_double), ("lambda2", C.c_double), ("theta", C.c_double),
                ("nu", C.c_double), ("eps", C.c_double), ("eps_tv_px", C.c_double),
                ("beta", C.c_double), ("sigma_g", C.c_double), ("sigma_d", C.c_double),
                ("Sigma", C.c_double), ("M", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("levels", C.c_int32), ("coarse_iters", C.c_int32), ("mixed_precision", C.c_int32),
                ("scaled", C.c_int32), ("coarse_rtol", C.c_double), ("smoother", C.c_int32),
                ("run_max", C.c_int32)]


class _Schedule(C.Structure):
    _fields_ = [("lds_side", C.c_int32), ("line_threads", C.c_int32), ("graph", C.c_int32),
                ("split_long", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("c1", C.c_double), ("c2", C.c_double), ("rel_res", C.c_double), ("res", C.c_double),
                ("res0", C.c_double), ("eta", C.c_double), ("cycles", C.c_int32), ("levels", C.c_int32),
                ("frac_fg", C.c_double), ("energy", C.c_double), ("frac_D", C.c_double),
                ("res_rows", C.c_double), ("res0_rows", C.c_double), ("rel_res_rows", C.c_double)]


@dataclass
class Params:
    model: int = 0
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
    levels: int = 0
    coarse_iters: int = 10
    mixed_precision: int = 1
    scaled: int = 1
    coarse_rtol: float = 1e-4
    smoother: int = 0           # 0 Hybrid Smoother 2, 1 GSLEX-I, 2 Hybrid Smoother 1, 3 GSLINE-I, 4 NEWT-I,
                                # 5 GSLEX-II, 6 GSLINE-II, 7 NEWT-II (Spencer-Chen)
    run_max: int = 0            # 0 maximal superpixel runs (the paper's); k > 0 runs cut into pieces of <= k

    def to_c(self) -> _Params:
        p = _Params()
        p.struct_size = C.sizeof(_Params)
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


# The global two-phase model (Chan-Vese, eq. cv / cvls) that the paper's
# methods also apply to, as a setting of the selective model: the edge weight
# w = g = 1/(1 + beta |grad|^2) is 1 everywhere at beta = 0, and theta = 0
# drops the selection (distance) term.  The paper gives no weights for it; mu =
# 0.05 at the default lambdas keeps the two-phase partition of a clean
# two-intensity image (at mu = 0.5 the one-phase state has the lower energy on
# such images of a few objects).
CHAN_VESE = {"model": 0, "beta": 0.0, "theta": 0.0, "mu": 0.05}


def chan_vese_params(**kw) -> Params:
    """Params of the global Chan-Vese workload (Spencer-Chen with w = 1 and no
    selection term); keyword arguments override."""
    return Params(**{**CHAN_VESE, **kw})


_lib = None


def lib():
    """Load the built library (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"libmgseg not built ({_build.LIB}); run __graft_entry__.build()")
        L = C.CDLL(_build.LIB)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.mgseg_params_default.argtypes = [C.POINTER(_Params)]
        L.mgseg_strerror.restype = C.c_char_p
        L.mgseg_strerror.argtypes = [C.c_int]
        L.mgseg_setup.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float), C.c_int,
                                  C.POINTER(_Params), vp, C.POINTER(vp)]
        L.mgseg_set_phi0.argtypes = [vp, vp, C.c_int]
        L.mgseg_vcycle.argtypes = [vp, dp]
        L.mgseg_solve.argtypes = [vp, C.c_double, C.c_int, ip, dp]
        L.mgseg_aos.argtypes = [vp, C.c_double, C.c_double, C.c_int, ip, dp, dp]
        L.mgseg_smoothing_rates.argtypes = [vp, C.c_int, dp, vp, C.c_int]
        L.mgseg_get_schedule.argtypes = [vp, C.POINTER(_Schedule)]
        L.mgseg_set_schedule.argtypes = [vp, C.POINTER(_Schedule)]
        L.mgseg_tune.argtypes = [vp, C.c_int, C.POINTER(_Schedule), dp]
        L.mgseg_get_phi.argtypes = [vp, vp, C.c_int]
        L.mgseg_get_mask.argtypes = [vp, vp, C.c_int]
        L.mgseg_get_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.mgseg_destroy.argtypes = [vp]
        L.mgseg_destroy.restype = None
        L.mgseg_level_shape.argtypes = [vp, C.c_int, ip, ip, dp]
        L.mgseg_debug_get.argtypes = [vp, C.c_int, C.c_int, vp]
        L.mgseg_debug_set.argtypes = [vp, C.c_int, C.c_int, vp]
        L.mgseg_debug_scalars.argtypes = [vp, dp]
        L.mgseg_debug_set_c.argtypes = [vp, C.c_double, C.c_double]
        L.mgseg_debug_op.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.mgseg_profile.argtypes = [vp, C.c_int, C.c_int]
        L.mgseg_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.mgseg_set_state.argtypes = [vp, vp, C.c_size_t]
        L.mgseg_profile_read.argtypes = [vp, C.c_int, dp, ip, dp]
        L.mgseg_setup_batch.argtypes = [C.c_int, C.POINTER(vp), ip, ip, ip, C.POINTER(C.POINTER(C.c_float)), ip,
                                        C.POINTER(_Params), vp, C.POINTER(vp)]
        L.mgseg_batch_tune.argtypes = [vp, C.c_int, ip, dp]
        L.mgseg_batch_set_streams.argtypes = [vp, C.c_int]
        L.mgseg_solve_batch.argtypes = [vp, C.c_double, C.c_int, ip, dp]
        L.mgseg_batch_ctx.argtypes = [vp, C.c_int, C.POINTER(vp)]
        L.mgseg_destroy_batch.argtypes = [vp]
        L.mgseg_destroy_batch.restype = None
        L.mgseg_net_create.argtypes = [C.c_int, C.c_int, C.c_uint64, C.POINTER(vp)]
        L.mgseg_net_forward.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_double, vp, vp]
        L.mgseg_net_backward.argtypes = [vp, vp, C.c_double, C.c_double, C.POINTER(C.c_float), vp]
        L.mgseg_net_adam_step.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double, vp]
        L.mgseg_net_param_count.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.mgseg_net_get_params.argtypes = [vp, vp, vp]
        L.mgseg_net_set_params.argtypes = [vp, vp]
        L.mgseg_net_get_adam.argtypes = [vp, vp, vp, C.POINTER(C.c_longlong)]
        L.mgseg_net_set_adam.argtypes = [vp, vp, vp, C.c_longlong]
        L.mgseg_net_destroy.argtypes = [vp]
        L.mgseg_net_destroy.restype = None
        L.mgseg_ctx_features.argtypes = [vp, vp]
        L.mgseg_net_profile.argtypes = [vp, C.c_int]
        L.mgseg_net_profile_read.argtypes = [vp, dp, ip, dp]
        L.mgseg_predict_phi0.argtypes = [vp, vp, C.c_double, ip]
        L.mgseg_reset_phi0.argtypes = [vp]
        L.mgseg_solve_noalloc.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float), C.c_int,
                                          C.POINTER(_Params), vp, C.c_double, C.c_int, vp, C.c_int, ip, dp]
        for name in ("mgseg_setup", "mgseg_set_phi0", "mgseg_vcycle", "mgseg_solve", "mgseg_get_phi",
                     "mgseg_get_mask", "mgseg_get_stats", "mgseg_level_shape", "mgseg_debug_get",
                     "mgseg_debug_set", "mgseg_debug_scalars", "mgseg_debug_set_c", "mgseg_debug_op",
                     "mgseg_profile", "mgseg_profile_read", "mgseg_setup_batch", "mgseg_batch_tune",
                     "mgseg_batch_set_streams", "mgseg_solve_batch", "mgseg_batch_ctx", "mgseg_net_create",
                     "mgseg_net_forward", "mgseg_net_backward", "mgseg_net_adam_step", "mgseg_net_param_count",
                     "mgseg_net_get_params", "mgseg_net_set_params", "mgseg_net_get_adam", "mgseg_net_set_adam",
                     "mgseg_ctx_features", "mgseg_predict_phi0",
                     "mgseg_reset_phi0", "mgseg_net_profile", "mgseg_net_profile_read",
                     "mgseg_get_state", "mgseg_set_state", "mgseg_solve_noalloc", "mgseg_aos",
                     "mgseg_smoothing_rates", "mgseg_get_schedule", "mgseg_set_schedule", "mgseg_tune"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code, where):
    if code != 0:
        raise MgsegError(code, where)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def solve_noalloc(image, markers, params: Params | None = None, tol=1e-6, max_cycles=50, stream=None,
                  out: torch.Tensor | None = None):
    """mgseg_solve_noalloc: setup, solve and the FP64 finest phi of one image with
    every device array in the library's static scratch (no device allocation
    inside the call).  out: an (n, m) float64 CUDA tensor to write (allocated here
    when None).  Returns (phi, cycles, rel, status)."""
    L = lib()
    params = params or Params()
    img = torch.as_tensor(image, dtype=torch.float32)
    if img.device.type != "cuda":
        img = img.to("cuda")
    img = img.contiguous()
    n, m = img.shape
    mk = np.ascontiguousarray(np.asarray(markers, np.float32).reshape(-1, 2))
    if out is None:
        out = torch.empty((n, m), dtype=torch.float64, device="cuda")
    p = params.to_c()
    cyc, rel = C.c_int(), C.c_double()
    code = L.mgseg_solve_noalloc(C.c_void_p(img.data_ptr()), n, m, m, mk.ctypes.data_as(C.POINTER(C.c_float)),
                                 len(mk), C.byref(p), _stream_ptr(stream), tol, max_cycles,
                                 C.c_void_p(out.data_ptr()), out.stride(0), C.byref(cyc), C.byref(rel))
    if code not in (0, 6):
        raise MgsegError(code, "mgseg_solve_noalloc")
    return out, cyc.value, rel.value, code


class Solver:
    """One image: setup, V-cycles, solve, results (all work on the GPU)."""

    def __init__(self, image, markers, params: Params | None = None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("mgseg needs a GPU (HIP device)")
        self.L = lib()
        self.params = params or Params()
        img = torch.as_tensor(image, dtype=torch.float32)
        if img.device.type != "cuda":
            img = img.to("cuda")
        img = img.contiguous()
        self.n, self.m = img.shape
        mk = np.ascontiguousarray(np.asarray(markers, np.float32).reshape(-1, 2))
        self._p = self.params.to_c()
        self.stream = stream or torch.cuda.current_stream()
        ctx = C.c_void_p()
        _check(self.L.mgseg_setup(C.c_void_p(img.data_ptr()), self.n, self.m, self.m,
                                  mk.ctypes.data_as(C.POINTER(C.c_float)), len(mk), C.byref(self._p),
                                  _stream_ptr(self.stream), C.byref(ctx)), "mgseg_setup")
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mgseg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vcycle(self) -> float:
        rel = C.c_double()
        _check(self.L.mgseg_vcycle(self.ctx, C.byref(rel)), "mgseg_vcycle")
        return rel.value

    def solve(self, tol=1e-6, max_cycles=50, raise_on_nonconv=False):
        cyc, rel = C.c_int(), C.c_double()
        code = self.L.mgseg_solve(self.ctx, tol, max_cycles, C.byref(cyc), C.byref(rel))
        if code not in (0, 6) or (code == 6 and raise_on_nonconv):
            raise MgsegError(code, "mgseg_solve")
        return cyc.value, rel.value, code == 0

    def aos(self, tau, eta_tol=1e-4, max_iters=200, raise_on_nonconv=False):
        """AOS steps (time step tau in units of h/mu) from the current phi until the
        relative change falls below eta_tol: (steps, last change, relative residual,
        reached)."""
        it, eta, rel = C.c_int(), C.c_double(), C.c_double()
        code = self.L.mgseg_aos(self.ctx, tau, eta_tol, max_iters, C.byref(it), C.byref(eta), C.byref(rel))
        if code not in (0, 6) or (code == 6 and raise_on_nonconv):
            raise MgsegError(code, "mgseg_aos")
        return it.value, eta.value, rel.value, code == 0

    def smoothing_rates(self, smoother, per_pixel=False):
        """Local Fourier analysis of a smoother at the current phi: (dict of mu~_max,
        mu~_avg, their values over the jump set and its share, per-pixel rates or None)."""
        out = (C.c_double * 5)()
        mu = torch.empty((self.n, self.m), dtype=torch.float32, device="cuda") if per_pixel else None
        _check(self.L.mgseg_smoothing_rates(self.ctx, smoother, out,
                                            C.c_void_p(mu.data_ptr()) if mu is not None else None, self.m),
               "mgseg_smoothing_rates")
        keys = ("mu_max", "mu_avg", "mu_max_D", "mu_avg_D", "share_D")
        return dict(zip(keys, list(out))), (mu.cpu().numpy() if mu is not None else None)

    def schedule(self) -> dict:
        sc = _Schedule()
        _check(self.L.mgseg_get_schedule(self.ctx, C.byref(sc)), "mgseg_get_schedule")
        return {k: getattr(sc, k) for k, _ in _Schedule._fields_}

    def set_schedule(self, lds_side=64, line_threads=0, graph=1, split_long=1):
        sc = _Schedule(lds_side, line_threads, graph, split_long)
        _check(self.L.mgseg_set_schedule(self.ctx, C.byref(sc)), "mgseg_set_schedule")

    def tune(self, trial_cycles=2):
        """Times every launch schedule from the current state and keeps the fastest
        (the state is restored): (schedule dict, ms per cycle)."""
        sc, ms = _Schedule(), C.c_double()
        _check(self.L.mgseg_tune(self.ctx, trial_cycles, C.byref(sc), C.byref(ms)), "mgseg_tune")
        return {k: getattr(sc, k) for k, _ in _Schedule._fields_}, ms.value

    def set_phi0(self, phi):
        t = torch.as_tensor(phi, dtype=torch.float32, device="cuda").contiguous()
        _check(self.L.mgseg_set_phi0(self.ctx, C.c_void_p(t.data_ptr()), self.m), "mgseg_set_phi0")

    def phi(self) -> torch.Tensor:
        out = torch.empty((self.n, self.m), dtype=torch.float64, device="cuda")
        _check(self.L.mgseg_get_phi(self.ctx, C.c_void_p(out.data_ptr()), self.m), "mgseg_get_phi")
        return out

    def mask(self) -> torch.Tensor:
        out = torch.empty((self.n, self.m), dtype=torch.uint8, device="cuda")
        _check(self.L.mgseg_get_mask(self.ctx, C.c_void_p(out.data_ptr()), self.m), "mgseg_get_mask")
        return out

    def stats(self) -> dict:
        s = _Stats()
        _check(self.L.mgseg_get_stats(self.ctx, C.byref(s)), "mgseg_get_stats")
        return {f[0]: getattr(s, f[0]) for f in _Stats._fields_}

    def features(self) -> torch.Tensor:
        """Network input of this image: [3, n, m] = (z, d, marker mask)."""
        out = torch.empty((3, self.n, self.m), dtype=torch.float32, device="cuda")
        _check(self.L.mgseg_ctx_features(self.ctx, C.c_void_p(out.data_ptr())), "mgseg_ctx_features")
        return out

    def predict_phi0(self, net: "Net", scale: float = 1.0) -> bool:
        """Start the solve from the network's phi0 (times scale) for this image
        if it holds every marker, else from the marker-based phi0; True if the
        network's phi0 was taken."""
        acc = C.c_int()
        _check(self.L.mgseg_predict_phi0(self.ctx, net.h, scale, C.byref(acc)), "mgseg_predict_phi0")
        return bool(acc.value)

    def reset_phi0(self):
        """Back to the marker-based initial level set of setup."""
        _check(self.L.mgseg_reset_phi0(self.ctx), "mgseg_reset_phi0")

    def get_state(self) -> bytes:
        """Checkpoint: the FP64 finest phi with the cycle counter and residual norms."""
        n = C.c_size_t(0)
        _check(self.L.mgseg_get_state(self.ctx, None, C.byref(n)), "mgseg_get_state")
        buf = C.create_string_buffer(n.value)
        _check(self.L.mgseg_get_state(self.ctx, buf, C.byref(n)), "mgseg_get_state")
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        """Resume from get_state() of a solve of the same image, markers and parameters."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(self.L.mgseg_set_state(self.ctx, buf, len(blob)), "mgseg_set_state")

    # ---- single steps (tests, profiling)
    def shape(self, level=0):
        n, m, h = C.c_int(), C.c_int(), C.c_double()
        _check(self.L.mgseg_level_shape(self.ctx, level, C.byref(n), C.byref(m), C.byref(h)), "level_shape")
        return n.value, m.value, h.value

    def get(self, name, level=0) -> np.ndarray:
        n, m, _ = self.shape(level)
        f = FIELD[name]
        dt = np.float64 if f in (8, 9) else (np.uint8 if f == 10 else np.float32)
        out = np.zeros((n, m), dt)
        _check(self.L.mgseg_debug_get(self.ctx, level, f, out.ctypes.data_as(C.c_void_p)), f"get {name}")
        return out

    def set(self, name, arr, level=0):
        n, m, _ = self.shape(level)
        f = FIELD[name]
        dt = np.float64 if f in (8, 9) else (np.uint8 if f == 10 else np.float32)
        a = np.ascontiguousarray(np.asarray(arr).reshape(n, m), dt)
        _check(self.L.mgseg_debug_set(self.ctx, level, f, a.ctypes.data_as(C.c_void_p)), f"set {name}")

    def scalars(self) -> dict:
        out = np.zeros(5)
        _check(self.L.mgseg_debug_scalars(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double))), "scalars")
        return dict(c1=out[0], c2=out[1], A1=out[2], res0=out[3], h0=out[4])

    def set_c(self, c1, c2):
        _check(self.L.mgseg_debug_set_c(self.ctx, c1, c2), "set_c")

    def profile(self, enable=True, kernel=0):
        _check(self.L.mgseg_profile(self.ctx, kernel, int(enable)), "profile")

    def profile_read(self, kernel=0):
        tot, cnt, by = C.c_double(), C.c_int(), C.c_double()
        _check(self.L.mgseg_profile_read(self.ctx, kernel, C.byref(tot), C.byref(cnt), C.byref(by)),
               "profile_read")
        return tot.value, cnt.value, by.value

    def op(self, name, level=0, arg=0):
        _check(self.L.mgseg_debug_op(self.ctx, level, OP[name], arg), f"op {name}")


class _View(Solver):
    """One image of a batch (the batch owns the context)."""

    def __init__(self, L, ctx, n, m, params):
        self.L, self.ctx, self.n, self.m, self.params = L, ctx, n, m, params

    def close(self):
        self.ctx = None


class Batch:
    """Images of uneven size solved together (mgseg_setup_batch): each image by
    its own context, V-cycles issued on internal streams, one wait per round."""

    def __init__(self, images, markers, params: Params | None = None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("mgseg needs a GPU (HIP device)")
        self.L = lib()
        self.params = params or Params()
        self._imgs = [torch.as_tensor(im, dtype=torch.float32).to("cuda").contiguous() for im in images]
        self._mk = [np.ascontiguousarray(np.asarray(mk, np.float32).reshape(-1, 2)) for mk in markers]
        cnt = len(self._imgs)
        vp = C.c_void_p
        imgs = (vp * cnt)(*[im.data_ptr() for im in self._imgs])
        ns = (C.c_int * cnt)(*[im.shape[0] for im in self._imgs])
        ms = (C.c_int * cnt)(*[im.shape[1] for im in self._imgs])
        mks = (C.POINTER(C.c_float) * cnt)(*[mk.ctypes.data_as(C.POINTER(C.c_float)) for mk in self._mk])
        ks = (C.c_int * cnt)(*[len(mk) for mk in self._mk])
        self._p = self.params.to_c()
        self.stream = stream or torch.cuda.current_stream()
        b = C.c_void_p()
        _check(self.L.mgseg_setup_batch(cnt, imgs, ns, ms, ms, mks, ks, C.byref(self._p), _stream_ptr(self.stream),
                                        C.byref(b)), "mgseg_setup_batch")
        self.b, self.count = b, cnt

    def tune(self, trial_rounds=1):
        s, ms = C.c_int(), C.c_double()
        _check(self.L.mgseg_batch_tune(self.b, trial_rounds, C.byref(s), C.byref(ms)), "mgseg_batch_tune")
        return s.value, ms.value

    def set_streams(self, n):
        _check(self.L.mgseg_batch_set_streams(self.b, n), "mgseg_batch_set_streams")

    def solve(self, tol=1e-6, max_cycles=50):
        cyc = (C.c_int * self.count)()
        rel = (C.c_double * self.count)()
        code = self.L.mgseg_solve_batch(self.b, tol, max_cycles, cyc, rel)
        if code not in (0, 6):
            raise MgsegError(code, "mgseg_solve_batch")
        return list(cyc), list(rel), code == 0

    def image(self, i) -> Solver:
        c = C.c_void_p()
        _check(self.L.mgseg_batch_ctx(self.b, i, C.byref(c)), "mgseg_batch_ctx")
        n, m = self._imgs[i].shape
        return _View(self.L, c, n, m, self.params)

    def close(self):
        if getattr(self, "b", None):
            self.L.mgseg_destroy_batch(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Warm-start network (mgseg_net_*): forward, backward, Adam, all on the GPU."""

    def __init__(self, base=16, depth=4, seed=0):
        if not torch.cuda.is_available():
            raise RuntimeError("mgseg needs a GPU (HIP device)")
        self.L = lib()
        self.base, self.depth = base, depth
        h = C.c_void_p()
        _check(self.L.mgseg_net_create(base, depth, seed, C.byref(h)), "mgseg_net_create")
        self.h = h
        cnt = C.c_longlong()
        _check(self.L.mgseg_net_param_count(self.h, C.byref(cnt)), "mgseg_net_param_count")
        self.count = cnt.value

    def forward(self, x: torch.Tensor, M: float, stream=None) -> torch.Tensor:
        """x [B, 3, H, W] FP32 on the device -> phi0 [B, H, W]."""
        x = x.to(device="cuda", dtype=torch.float32).contiguous()
        B, ch, H, W = x.shape
        if ch != 3:
            raise ValueError("the network takes 3 input channels")
        out = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
        self._keep = x
        _check(self.L.mgseg_net_forward(self.h, C.c_void_p(x.data_ptr()), B, H, W, M, C.c_void_p(out.data_ptr()),
                                        _stream_ptr(stream)), "mgseg_net_forward")
        return out

    def backward(self, target: torch.Tensor, M: float, pos_weight: float = 1.0, stream=None) -> float:
        t = target.to(device="cuda", dtype=torch.float32).contiguous()
        loss = C.c_float()
        _check(self.L.mgseg_net_backward(self.h, C.c_void_p(t.data_ptr()), M, pos_weight, C.byref(loss),
                                         _stream_ptr(stream)), "mgseg_net_backward")
        return loss.value

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        _check(self.L.mgseg_net_adam_step(self.h, lr, b1, b2, eps, _stream_ptr(stream)), "mgseg_net_adam_step")

    def params(self):
        """(values, gradients) as FP32 host arrays in the library's order."""
        p, g = np.zeros(self.count, np.float32), np.zeros(self.count, np.float32)
        _check(self.L.mgseg_net_get_params(self.h, p.ctypes.data_as(C.c_void_p), g.ctypes.data_as(C.c_void_p)),
               "mgseg_net_get_params")
        return p, g

    def set_params(self, values):
        v = np.ascontiguousarray(values, np.float32)
        if v.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {v.size}")
        _check(self.L.mgseg_net_set_params(self.h, v.ctypes.data_as(C.c_void_p)), "mgseg_net_set_params")

    def adam_state(self):
        """(first moments, second moments, steps taken) of Adam, host arrays in the parameter order."""
        m, v, t = np.zeros(self.count, np.float32), np.zeros(self.count, np.float32), C.c_longlong()
        _check(self.L.mgseg_net_get_adam(self.h, m.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                         C.byref(t)), "mgseg_net_get_adam")
        return m, v, t.value

    def set_adam_state(self, m, v, steps):
        m, v = np.ascontiguousarray(m, np.float32), np.ascontiguousarray(v, np.float32)
        if m.size != self.count or v.size != self.count:
            raise ValueError(f"expected {self.count} moments each, got {m.size} and {v.size}")
        _check(self.L.mgseg_net_set_adam(self.h, m.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                         int(steps)), "mgseg_net_set_adam")

    def profile(self, enable=True):
        """Time every convolution launch with HIP events (clears the record)."""
        _check(self.L.mgseg_net_profile(self.h, int(enable)), "mgseg_net_profile")

    def profile_read(self):
        """(summed convolution launch time in ms, launches, algorithmic flops)."""
        ms, n, fl = C.c_double(), C.c_int(), C.c_double()
        _check(self.L.mgseg_net_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(fl)), "mgseg_net_profile_read")
        return ms.value, n.value, fl.value

    def close(self):
        if getattr(self, "h", None):
            self.L.mgseg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
