"""MI355X-native AB-/BA-GKB for X-ray CT with an unmatched back projector.

A thin ctypes binding over ``libgkb.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/gkb.h``).  The binding only marshals arguments: tensors are
allocated by PyTorch on the GPU and their device pointers are handed to the
library together with the current HIP stream; every step of the projectors
and of the GKB iteration runs in the library's kernels.

There is no CPU fallback: if ``libgkb.so`` has not been built, importing the
binding raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import synth  # noqa: F401  (seeded input generators)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgkb.so")

GKB_OK, GKB_EINVAL, GKB_ENOMEM, GKB_EDEVICE, GKB_ENONFINITE, GKB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STOP_NONE, STOP_DP, STOP_KMAX, STOP_BREAKDOWN, STOP_DP_NOT_REACHED, STOP_FALLBACK, STOP_RNS = 0, 1, 2, 3, 4, 5, 6
GKB_PAR2D, GKB_FAN2D, GKB_CONE3D = 0, 1, 2
GKB_F32, GKB_F64 = 0, 1
GKB_METHOD_AB, GKB_METHOD_BA = 0, 1
GKB_BATCH_LAUNCHES, GKB_BATCH_GRAPH = 0, 1
GKB_LAMBDA_FIXED, GKB_LAMBDA_DP, GKB_LAMBDA_GCV = 0, 1, 2

STATUS_NAMES = {0: "GKB_OK", -1: "GKB_EINVAL", -2: "GKB_ENOMEM", -3: "GKB_EDEVICE", -4: "GKB_ENONFINITE",
                -5: "GKB_EUNSUPPORTED"}
EXPORTED = ("gkb_create", "gkb_destroy", "gkb_set_stream", "gkb_last_error", "gkb_forward", "gkb_back",
            "gkb_forward_adjoint", "gkb_back_adjoint", "gkb_ab_solve", "gkb_ba_solve", "gkb_gkb_solve",
            "gkb_batch_solve", "gkb_trace_enable", "gkb_trace_only", "gkb_trace_reset", "gkb_trace_get", "gkb_net_create",
            "gkb_net_destroy", "gkb_net_set_weights", "gkb_net_get_weights", "gkb_net_save", "gkb_net_load",
            "gkb_net_apply", "gkb_net_frozen_apply", "gkb_net_grad", "gkb_net_train_step", "gkb_back_noalloc",
            "gkb_check_geometry", "gkb_ab_gmres_solve", "gkb_ba_gmres_solve", "gkb_set_batch_mode",
            "gkb_autotune", "gkb_set_tuning", "gkb_ab_hybrid_solve", "gkb_ba_hybrid_solve")
NET_PARAMS = 19008
GKB_NET_FBP, GKB_NET_FROZEN = 0, 1


class GkbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_views", ctypes.c_int), ("angles", ctypes.POINTER(ctypes.c_double)),
                ("angle_span", ctypes.c_double), ("n_det_u", ctypes.c_int), ("n_det_v", ctypes.c_int),
                ("det_pitch_u", ctypes.c_double), ("det_pitch_v", ctypes.c_double),
                ("src_dist", ctypes.c_double), ("src_det_dist", ctypes.c_double)]


class HybridOpts(ctypes.Structure):
    _fields_ = [("lambda_rule", ctypes.c_int), ("tau_proj", ctypes.c_double), ("eta_proj", ctypes.c_double),
                ("tsvd_rank", ctypes.c_int), ("lambda_history", ctypes.POINTER(ctypes.c_double))]


class SolveOpts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("lam", ctypes.c_double), ("use_dp", ctypes.c_int),
                ("tau", ctypes.c_double), ("noise_norm", ctypes.c_double), ("reorth", ctypes.c_int),
                ("precond", ctypes.c_void_p), ("residual_history", ctypes.POINTER(ctypes.c_double)),
                ("alpha_history", ctypes.POINTER(ctypes.c_double)),
                ("t_history", ctypes.POINTER(ctypes.c_double)), ("rns_eps", ctypes.c_double),
                ("x_true", ctypes.c_void_p), ("rre_history", ctypes.POINTER(ctypes.c_double))]


class CheckStats(ctypes.Structure):
    _fields_ = [("units", ctypes.c_longlong), ("reads", ctypes.c_longlong), ("out_of_bounds", ctypes.c_longlong),
                ("uncovered", ctypes.c_longlong), ("max_uncovered_weight", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("at_views_per_step", ctypes.c_int), ("b_views_per_step", ctypes.c_int),
                ("at_us", ctypes.c_double * 3), ("b_us", ctypes.c_double * 2)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("k_stop", ctypes.c_int), ("reason", ctypes.c_int), ("residual", ctypes.c_double),
                ("proj_residual", ctypes.c_double), ("t1", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("seconds", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgkb.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2606_31153_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, cp = ctypes.c_void_p, ctypes.c_int
        G = ctypes.POINTER(Geometry)
        L.gkb_create.argtypes = [ctypes.POINTER(vp), cp, vp]
        L.gkb_destroy.argtypes = [vp]
        L.gkb_destroy.restype = None
        L.gkb_set_stream.argtypes = [vp, vp]
        L.gkb_last_error.restype = ctypes.c_char_p
        for name in ("gkb_forward", "gkb_back", "gkb_forward_adjoint", "gkb_back_adjoint", "gkb_back_noalloc"):
            getattr(L, name).argtypes = [vp, G, cp, vp, vp]
        for name in ("gkb_ab_solve", "gkb_ba_solve", "gkb_gkb_solve", "gkb_ab_gmres_solve", "gkb_ba_gmres_solve"):
            getattr(L, name).argtypes = [vp, G, cp, vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo)]
        for name in ("gkb_ab_hybrid_solve", "gkb_ba_hybrid_solve"):
            getattr(L, name).argtypes = [vp, G, cp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(HybridOpts), vp,
                                         ctypes.POINTER(SolveInfo)]
        L.gkb_batch_solve.argtypes = [vp, cp, cp, G, cp, ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                                      ctypes.POINTER(vp), ctypes.POINTER(SolveInfo)]
        L.gkb_net_create.argtypes = [vp, ctypes.POINTER(vp), cp, cp, cp, ctypes.c_ulonglong]
        L.gkb_net_destroy.argtypes = [vp]
        L.gkb_net_destroy.restype = None
        FP = ctypes.POINTER(ctypes.c_float)
        L.gkb_net_set_weights.argtypes = [vp, FP, ctypes.c_longlong]
        L.gkb_net_get_weights.argtypes = [vp, FP, ctypes.c_longlong]
        L.gkb_net_save.argtypes = [vp, ctypes.c_char_p]
        L.gkb_net_load.argtypes = [vp, ctypes.c_char_p]
        L.gkb_net_apply.argtypes = [vp, vp, G, vp, vp]
        L.gkb_net_frozen_apply.argtypes = [vp, vp, G, vp, vp, vp, cp]
        L.gkb_net_grad.argtypes = [vp, vp, G, cp, vp, vp, cp, ctypes.POINTER(ctypes.c_double), FP]
        L.gkb_net_train_step.argtypes = [vp, vp, G, cp, vp, vp, cp, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_double)]
        L.gkb_check_geometry.argtypes = [G, cp, cp, ctypes.POINTER(CheckStats), ctypes.POINTER(cp)]
        L.gkb_set_batch_mode.argtypes = [vp, cp]
        L.gkb_autotune.argtypes = [vp, G, cp, ctypes.POINTER(Tuning)]
        L.gkb_set_tuning.argtypes = [vp, G, cp, ctypes.POINTER(Tuning)]
        L.gkb_trace_enable.argtypes = [vp, cp]
        L.gkb_trace_only.argtypes = [vp, ctypes.c_char_p]
        L.gkb_trace_reset.argtypes = [vp]
        L.gkb_trace_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(cp), ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _check(status: int):
    if status != GKB_OK:
        raise GkbError(status, lib().gkb_last_error().decode())


def make_geometry(geom) -> tuple:
    """C geometry struct from ``synth.Geometry``; returns (struct, keep-alive)."""
    keep = []
    g = Geometry()
    g.kind, g.nx, g.ny, g.nz = geom.kind, geom.nx, geom.ny, geom.nz
    g.n_views = geom.n_views
    if geom.angles is not None:
        a = np.ascontiguousarray(geom.angles, dtype=np.float64)
        keep.append(a)
        g.angles = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g.angle_span = geom.angle_span
    g.n_det_u, g.n_det_v = geom.n_det_u, geom.n_det_v
    g.det_pitch_u, g.det_pitch_v = geom.det_pitch_u, geom.det_pitch_v
    g.src_dist, g.src_det_dist = geom.src_dist, geom.src_det_dist
    return g, keep


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return GKB_F32
    if t.dtype == torch.float64:
        return GKB_F64
    raise TypeError("tensors must be float32 or float64")


def _dev_ptr(t, numel: int):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.numel() != numel:
        raise ValueError("tensor has %d elements, expected %d" % (t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A gkb_ctx bound to one GPU; launches on PyTorch's current stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        import torch
        self.device = device
        if stream is None:
            with torch.cuda.device(device):
                stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib().gkb_create(ctypes.byref(h), device, ctypes.c_void_p(stream)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().gkb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_batch_mode(self, mode: int):
        """GKB_BATCH_LAUNCHES or GKB_BATCH_GRAPH for gkb_batch_solve."""
        _check(lib().gkb_set_batch_mode(self.handle, mode))

    def set_stream(self, stream: int):
        _check(lib().gkb_set_stream(self.handle, ctypes.c_void_p(stream)))

    # ---- tracing ----
    def trace_enable(self, on: bool = True):
        _check(lib().gkb_trace_enable(self.handle, 1 if on else 0))

    def trace_only(self, kernel: Optional[str]):
        """Record only `kernel` while tracing (None: every kernel)."""
        _check(lib().gkb_trace_only(self.handle, kernel.encode() if kernel else None))

    def trace_reset(self):
        _check(lib().gkb_trace_reset(self.handle))

    def trace_get(self, kernel: str):
        cnt = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().gkb_trace_get(self.handle, kernel.encode(), ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value


def _proj(name: str, ctx: Context, geom, inp, out, n_in: int, n_out: int):
    g, keep = make_geometry(geom)
    code = _dtype_code(inp)
    if out.dtype != inp.dtype:
        raise TypeError("input and output dtypes differ")
    _check(getattr(lib(), name)(ctx.handle, ctypes.byref(g), code, _dev_ptr(inp, n_in), _dev_ptr(out, n_out)))
    return out


def gkb_forward(ctx: Context, geom, x, y):
    """y = A x (Joseph forward projector)."""
    return _proj("gkb_forward", ctx, geom, x, y, geom.n, geom.m)


def gkb_back(ctx: Context, geom, y, x):
    """x = B y (pixel-driven back projector)."""
    return _proj("gkb_back", ctx, geom, y, x, geom.m, geom.n)


def gkb_back_noalloc(ctx: Context, geom, y, x):
    """x = B y with no device allocation (scratch in the library's fixed
    device array; overlapping calls on one GPU race)."""
    return _proj("gkb_back_noalloc", ctx, geom, y, x, geom.m, geom.n)


def gkb_forward_adjoint(ctx: Context, geom, y, x):
    """x = A^T y (exact transpose of A)."""
    return _proj("gkb_forward_adjoint", ctx, geom, y, x, geom.m, geom.n)


def gkb_back_adjoint(ctx: Context, geom, x, y):
    """y = B^T x (exact transpose of B)."""
    return _proj("gkb_back_adjoint", ctx, geom, x, y, geom.n, geom.m)


def gkb_check_geometry(geom, dtype_code: int = GKB_F32, stride: int = 1):
    """Host replay of the projector kernels' address arithmetic for ``geom``
    (no GPU): ({"A"|"B"|"At"|"Bt": CheckStats}, orders_ok)."""
    g, keep = make_geometry(geom)
    st = (CheckStats * 4)()
    ok = ctypes.c_int()
    _check(lib().gkb_check_geometry(ctypes.byref(g), dtype_code, stride, st, ctypes.byref(ok)))
    return dict(zip(("A", "B", "At", "Bt"), st)), bool(ok.value)


def gkb_autotune(ctx: Context, geom, dtype_code: int = GKB_F32) -> Tuning:
    """Times the launch choices of geom on the device and keeps the fastest."""
    g, keep = make_geometry(geom)
    t = Tuning()
    _check(lib().gkb_autotune(ctx.handle, ctypes.byref(g), dtype_code, ctypes.byref(t)))
    return t


def gkb_set_tuning(ctx: Context, geom, at_views: int, b_views: int, dtype_code: int = GKB_F32) -> None:
    g, keep = make_geometry(geom)
    t = Tuning()
    t.at_views_per_step, t.b_views_per_step = at_views, b_views
    _check(lib().gkb_set_tuning(ctx.handle, ctypes.byref(g), dtype_code, ctypes.byref(t)))


@dataclass
class SolveResult:
    k_stop: int
    reason: int
    residual: float
    proj_residual: float
    t1: float
    alpha1: float
    seconds: float
    rho: np.ndarray
    alpha: np.ndarray
    t: np.ndarray
    rre: Optional[np.ndarray] = None  # RRE(x_k), k = 1..k_stop, when x_true was given
    lam: Optional[np.ndarray] = None  # lambda_k, k = 1..k_stop (hybrid solves)


def _solve(name: str, ctx: Context, geom, b, x, k_max: int, lam: float = 0.0, use_dp: bool = False,
           tau: float = 1.0, noise_norm: float = 0.0, reorth: bool = True, precond=None,
           rns_eps: float = 0.0, x_true=None, hybrid: Optional[HybridOpts] = None) -> SolveResult:
    g, keep = make_geometry(geom)
    code = _dtype_code(b)
    if x.dtype != b.dtype:
        raise TypeError("b and x dtypes differ")
    rho = np.zeros(max(k_max, 1))
    alpha = np.zeros(k_max + 1)
    t = np.zeros(k_max + 1)
    P = ctypes.POINTER(ctypes.c_double)
    rre = None
    if x_true is not None:
        if x_true.dtype != b.dtype:
            raise TypeError("x_true and b dtypes differ")
        rre = np.zeros(max(k_max, 1))
    o = SolveOpts(k_max, lam, 1 if use_dp else 0, tau, noise_norm, 1 if reorth else 0,
                  None if precond is None else precond.handle,
                  rho.ctypes.data_as(P), alpha.ctypes.data_as(P), t.ctypes.data_as(P), rns_eps,
                  None if x_true is None else _dev_ptr(x_true, geom.n).value,
                  None if rre is None else rre.ctypes.data_as(P))
    info = SolveInfo()
    extra = () if hybrid is None else (ctypes.byref(hybrid),)
    _check(getattr(lib(), name)(ctx.handle, ctypes.byref(g), code, _dev_ptr(b, geom.m), ctypes.byref(o), *extra,
                                _dev_ptr(x, geom.n), ctypes.byref(info)))
    k = info.k_stop
    return SolveResult(k_stop=k, reason=info.reason, residual=info.residual, proj_residual=info.proj_residual,
                       t1=info.t1, alpha1=info.alpha1, seconds=info.seconds, rho=rho[:k], alpha=alpha[:k + 1],
                       t=t[:k + 1], rre=None if rre is None else rre[:k])


def gkb_ab_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """AB-GKB: GKB on M = AB from b; x = B Q_k u_k."""
    return _solve("gkb_ab_solve", ctx, geom, b, x, k_max, **kw)


def gkb_ba_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """BA-GKB: GKB on M = BA from B b; x = Q_k u_k."""
    return _solve("gkb_ba_solve", ctx, geom, b, x, k_max, **kw)


def gkb_gkb_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """Matched GKB (B := A^T), equivalent to LSQR."""
    return _solve("gkb_gkb_solve", ctx, geom, b, x, k_max, **kw)


def gkb_ab_gmres_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """AB-GMRES (B as right preconditioner): x = B Q_k u_k.  ``alpha`` holds
    ||r_0|| then h_{k+1,k}; ``t`` is zero."""
    return _solve("gkb_ab_gmres_solve", ctx, geom, b, x, k_max, **kw)


def gkb_ba_gmres_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """BA-GMRES (B as left preconditioner): x = Q_k u_k."""
    return _solve("gkb_ba_gmres_solve", ctx, geom, b, x, k_max, **kw)


def _hybrid(name: str, ctx: Context, geom, b, x, k_max: int, rule: int = GKB_LAMBDA_FIXED, tau_proj: float = 1.0,
            eta_proj: float = 0.0, tsvd_rank: int = 0, **kw) -> SolveResult:
    lam = np.zeros(max(k_max, 1))
    h = HybridOpts(rule, tau_proj, eta_proj, tsvd_rank, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    r = _solve(name, ctx, geom, b, x, k_max, hybrid=h, **kw)
    r.lam = lam[:r.k_stop] if rule != GKB_LAMBDA_FIXED else None
    return r


def gkb_ab_hybrid_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """Hybrid AB-GKB (rule GKB_LAMBDA_DP with tau_proj, eta_proj = ||e||, or
    GKB_LAMBDA_GCV), or the enlarged-subspace TSVD (tsvd_rank)."""
    return _hybrid("gkb_ab_hybrid_solve", ctx, geom, b, x, k_max, **kw)


def gkb_ba_hybrid_solve(ctx: Context, geom, b, x, k_max: int, **kw) -> SolveResult:
    """Hybrid BA-GKB (rule GKB_LAMBDA_DP with eta_proj = ||B e||, or
    GKB_LAMBDA_GCV), or the enlarged-subspace TSVD (tsvd_rank)."""
    return _hybrid("gkb_ba_hybrid_solve", ctx, geom, b, x, k_max, **kw)


def _opts(k_max: int, lam: float = 0.0, use_dp: bool = False, tau: float = 1.0, noise_norm: float = 0.0,
          reorth: bool = True, rns_eps: float = 0.0):
    """(SolveOpts, history arrays) for one problem."""
    rho = np.zeros(max(k_max, 1))
    alpha = np.zeros(k_max + 1)
    t = np.zeros(k_max + 1)
    P = ctypes.POINTER(ctypes.c_double)
    o = SolveOpts(k_max, lam, 1 if use_dp else 0, tau, noise_norm, 1 if reorth else 0, None,
                  rho.ctypes.data_as(P), alpha.ctypes.data_as(P), t.ctypes.data_as(P), rns_eps)
    return o, (rho, alpha, t)


def gkb_batch_solve(ctx: Context, method: int, geoms, bs, xs, opts) -> list:
    """Batched solve of independent slices (AB-GKB or BA-GKB per ``method``):
    ``geoms``, ``bs``, ``xs`` are per-slice geometries and device tensors;
    ``opts`` is a list of per-slice keyword dicts (k_max, lam, use_dp, tau,
    noise_norm, reorth, rns_eps).  Returns one SolveResult per slice."""
    ns = len(geoms)
    if not (len(bs) == len(xs) == len(opts) == ns):
        raise ValueError("geoms, bs, xs and opts must have one entry per slice")
    G = (Geometry * ns)()
    O = (SolveOpts * ns)()
    I = (SolveInfo * ns)()
    Bp = (ctypes.c_void_p * ns)()
    Xp = (ctypes.c_void_p * ns)()
    keep, hist = [], []
    code = None
    for s in range(ns):
        g, k = make_geometry(geoms[s])
        keep.append(k)
        G[s] = g
        o, h = _opts(**opts[s])
        O[s] = o
        hist.append(h)
        c = _dtype_code(bs[s])
        if code is None:
            code = c
        if c != code or xs[s].dtype != bs[s].dtype:
            raise TypeError("all slices must share one dtype")
        Bp[s] = _dev_ptr(bs[s], geoms[s].m).value
        Xp[s] = _dev_ptr(xs[s], geoms[s].n).value
    if code is None:  # no slices: the library reports the invalid count
        code = GKB_F32
    _check(lib().gkb_batch_solve(ctx.handle, method, ns, G, code, Bp, O, Xp, I))
    out = []
    for s in range(ns):
        rho, alpha, t = hist[s]
        k = I[s].k_stop
        out.append(SolveResult(k_stop=k, reason=I[s].reason, residual=I[s].residual,
                               proj_residual=I[s].proj_residual, t1=I[s].t1, alpha1=I[s].alpha1,
                               seconds=I[s].seconds, rho=rho[:k], alpha=alpha[:k + 1], t=t[:k + 1]))
    return out


class Net:
    """The learned sinogram filter (gkb_net): 32 channels, kernel 9, 4 layers,
    He-initialised from ``seed``; lives on the context's device."""

    def __init__(self, ctx: Context, seed: int = 0, channels: int = 32, ksize: int = 9, layers: int = 4):
        h = ctypes.c_void_p()
        _check(lib().gkb_net_create(ctx.handle, ctypes.byref(h), channels, ksize, layers, seed))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().gkb_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self) -> np.ndarray:
        w = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(lib().gkb_net_get_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))
        return w

    def set_weights(self, w) -> None:
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        _check(lib().gkb_net_set_weights(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))

    def save(self, path: str) -> None:
        _check(lib().gkb_net_save(self.handle, path.encode()))

    def load(self, path: str) -> None:
        _check(lib().gkb_net_load(self.handle, path.encode()))


def gkb_net_apply(ctx: Context, net: Net, geom, y, out):
    """out = N(y) (FP32 device tensors of m elements)."""
    g, keep = make_geometry(geom)
    _check(lib().gkb_net_apply(ctx.handle, net.handle, ctypes.byref(g), _dev_ptr(y, geom.m), _dev_ptr(out, geom.m)))
    return out


def gkb_net_frozen_apply(ctx: Context, net: Net, geom, b, y, out, transpose: bool = False):
    """out = F y or F^T y with the masks of b frozen."""
    g, keep = make_geometry(geom)
    _check(lib().gkb_net_frozen_apply(ctx.handle, net.handle, ctypes.byref(g), _dev_ptr(b, geom.m),
                                      _dev_ptr(y, geom.m), _dev_ptr(out, geom.m), 1 if transpose else 0))
    return out


def gkb_net_grad(ctx: Context, net: Net, geom, bs, xs, objective: int = GKB_NET_FBP):
    """(mean loss, gradient [19008]) for a batch: bs [batch, m], xs [batch, n] FP32 device tensors."""
    g, keep = make_geometry(geom)
    batch = bs.shape[0]
    loss = ctypes.c_double()
    grad = np.zeros(NET_PARAMS, dtype=np.float32)
    _check(lib().gkb_net_grad(ctx.handle, net.handle, ctypes.byref(g), batch, _dev_ptr(bs, batch * geom.m),
                              _dev_ptr(xs, batch * geom.n), objective, ctypes.byref(loss),
                              grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return loss.value, grad


def gkb_net_train_step(ctx: Context, net: Net, geom, bs, xs, lr: float, objective: int = GKB_NET_FBP) -> float:
    """One Adam step on a batch; returns the batch loss before the step."""
    g, keep = make_geometry(geom)
    batch = bs.shape[0]
    loss = ctypes.c_double()
    _check(lib().gkb_net_train_step(ctx.handle, net.handle, ctypes.byref(g), batch, _dev_ptr(bs, batch * geom.m),
                                    _dev_ptr(xs, batch * geom.n), objective, lr, ctypes.byref(loss)))
    return loss.value
