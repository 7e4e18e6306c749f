"""FP64 CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; it
shares no code with it.  The only module both sides use is the seeded input
generator ``paper_2606_31153_amd.synth``, which holds none of the method's
arithmetic.

``oracle.c`` (ctypes) holds the projectors, the GKB driver and the Jacobi
SVD; ``dense.py`` holds an independent NumPy builder of the dense projector
matrices from their weight formulas (a second implementation for tiny
sizes); ``learned.py`` holds the learned-preconditioner reference;
``hybrid.py`` holds hybrid regularisation (lambda_k chosen on the projected
problem) and the enlarged-subspace TSVD on top of the GKB driver.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KIND = {0: 0, 1: 1, 2: 2}
OR_DENSE = 9
MODE_AB, MODE_BA, MODE_GKB = 0, 1, 2
STOP_DP, STOP_KMAX, STOP_BREAKDOWN, STOP_DP_NOT_REACHED, STOP_RNS = 1, 2, 3, 4, 6


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("nv", ctypes.c_int), ("nu", ctypes.c_int), ("nw", ctypes.c_int),
                ("du", ctypes.c_double), ("dw", ctypes.c_double), ("D", ctypes.c_double),
                ("SDD", ctypes.c_double), ("ang", ctypes.POINTER(ctypes.c_double)),
                ("dm", ctypes.c_int), ("dn", ctypes.c_int),
                ("dA", ctypes.POINTER(ctypes.c_double)), ("dB", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("lam", ctypes.c_double), ("use_dp", ctypes.c_int),
                ("tau", ctypes.c_double), ("noise_norm", ctypes.c_double), ("reorth", ctypes.c_int),
                ("rns_eps", ctypes.c_double), ("xtrue", ctypes.c_void_p), ("rre", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("k_stop", ctypes.c_int), ("reason", ctypes.c_int), ("residual", ctypes.c_double),
                ("proj_residual", ctypes.c_double), ("t1", ctypes.c_double), ("alpha1", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(ctypes.c_double)
        G = ctypes.POINTER(_Geom)
        for name in ("or_forward", "or_forward_adjoint", "or_back", "or_back_adjoint"):
            f = getattr(L, name)
            f.argtypes = [G, P, P]
            f.restype = None
        L.or_gkb.argtypes = [G, ctypes.c_int, P, ctypes.POINTER(_Opts), P, P, P, P, P, P, P, P,
                             ctypes.POINTER(_Info)]
        L.or_gkb.restype = ctypes.c_int
        L.or_gmres.argtypes = [G, ctypes.c_int, P, ctypes.POINTER(_Opts), P, P, P, P, P, ctypes.POINTER(_Info)]
        L.or_gmres.restype = ctypes.c_int
        L.or_proj_solve.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P, P, P]
        L.or_proj_solve.restype = None
        L.or_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        L.or_jacobi_svd.restype = ctypes.c_int
        for name in ("or_cone_forward_sampled", "or_cone_back_sampled", "or_cone_back_adjoint_sampled",
                     "or_cone_forward_adjoint_sampled"):
            f = getattr(L, name)
            f.argtypes = [G, P, ctypes.POINTER(ctypes.c_longlong), ctypes.c_longlong, P]
            f.restype = ctypes.c_int
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Operator:
    """A projector pair (A, B) and its exact transposes, in FP64 on the CPU.

    Either a geometry (``paper_2606_31153_amd.synth.Geometry``) or explicit
    dense matrices A (m x n) and B (n x m)."""

    def __init__(self, geom=None, A: Optional[np.ndarray] = None, B: Optional[np.ndarray] = None):
        self._keep = []
        g = _Geom()
        if geom is not None:
            ang = np.ascontiguousarray(geom.view_angles(), dtype=np.float64)
            self._keep.append(ang)
            g.kind = KIND[geom.kind]
            g.nx, g.ny, g.nz = geom.nx, geom.ny, geom.nz
            g.nv, g.nu, g.nw = geom.n_views, geom.n_det_u, geom.n_det_v
            g.du, g.dw = geom.det_pitch_u, geom.det_pitch_v
            g.D, g.SDD = geom.src_dist, geom.src_det_dist
            g.ang = _ptr(ang)
            self.m, self.n = geom.m, geom.n
            self.image_shape, self.sino_shape = geom.image_shape(), geom.sino_shape()
        else:
            A = np.ascontiguousarray(A, dtype=np.float64)
            B = np.ascontiguousarray(B, dtype=np.float64)
            assert B.shape == (A.shape[1], A.shape[0])
            self._keep += [A, B]
            g.kind = OR_DENSE
            g.dm, g.dn = A.shape
            g.dA, g.dB = _ptr(A), _ptr(B)
            self.m, self.n = A.shape
            self.image_shape, self.sino_shape = (self.n,), (self.m,)
        self.g = g

    def _call(self, name, inp, out_size, out_shape):
        a = np.ascontiguousarray(np.asarray(inp, dtype=np.float64).reshape(-1))
        out = np.zeros(out_size, dtype=np.float64)
        getattr(lib(), name)(ctypes.byref(self.g), _ptr(a), _ptr(out))
        return out.reshape(out_shape)

    def A(self, x):
        return self._call("or_forward", x, self.m, self.sino_shape)

    def _sampled(self, name, inp, ids, size):
        a = np.ascontiguousarray(np.asarray(inp, dtype=np.float64).reshape(-1))
        assert a.size == size
        idx = np.ascontiguousarray(np.asarray(ids, dtype=np.int64).reshape(-1))
        out = np.zeros(idx.size, dtype=np.float64)
        rc = getattr(lib(), name)(ctypes.byref(self.g), _ptr(a),
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), idx.size, _ptr(out))
        if rc != 0:
            raise ValueError("%s: not a cone-beam geometry or index out of range" % name)
        return out

    def A_at(self, x, ray_ids):
        """(A x) at the listed detector pixels (cone beam only)."""
        return self._sampled("or_cone_forward_sampled", x, ray_ids, self.n)

    def B_at(self, y, voxel_ids):
        """(B y) at the listed voxels (cone beam only)."""
        return self._sampled("or_cone_back_sampled", y, voxel_ids, self.m)

    def At_at(self, y, voxel_ids):
        """(A^T y) at the listed voxels (cone beam only)."""
        return self._sampled("or_cone_forward_adjoint_sampled", y, voxel_ids, self.m)

    def Bt_at(self, x, ray_ids):
        """(B^T x) at the listed detector pixels (cone beam only)."""
        return self._sampled("or_cone_back_adjoint_sampled", x, ray_ids, self.n)

    def At(self, y):
        return self._call("or_forward_adjoint", y, self.n, self.image_shape)

    def B(self, y):
        return self._call("or_back", y, self.n, self.image_shape)

    def Bt(self, x):
        return self._call("or_back_adjoint", x, self.m, self.sino_shape)


@dataclass
class GKBResult:
    x: np.ndarray
    k_stop: int
    reason: int
    residual: float
    proj_residual: float
    t1: float
    alpha1: float
    rho: np.ndarray
    pres: np.ndarray
    alpha: np.ndarray
    t: np.ndarray
    Q: Optional[np.ndarray] = None
    S: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    rre: Optional[np.ndarray] = None


def gkb(op: Operator, mode: int, b, k_max: int, lam: float = 0.0, use_dp: bool = False, tau: float = 1.0,
        noise_norm: float = 0.0, reorth: int = 1, want_bases: bool = False, rns_eps: float = 0.0,
        x_true=None) -> GKBResult:
    """AB-GKB (mode 0), BA-GKB (mode 1) or matched GKB (mode 2).  Stops by the
    discrepancy principle (use_dp), residual norm stagnation (rns_eps > 0,
    eq. RNS: the first k >= 2 whose residual changed by less than rns_eps
    relative to the previous one; x_k is returned), breakdown or k_max.
    With x_true, ``rre`` holds RRE(x_k) = ||x_k - x_true|| / ||x_true|| (eq. RE)
    for k = 1..k_stop."""
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    assert b.size == op.m
    xt = None if x_true is None else np.ascontiguousarray(np.asarray(x_true, dtype=np.float64).reshape(-1))
    assert xt is None or xt.size == op.n
    rre = np.zeros(k_max)
    o = _Opts(k_max, lam, 1 if use_dp else 0, tau, noise_norm, reorth, rns_eps,
              None if xt is None else xt.ctypes.data, None if xt is None else rre.ctypes.data)
    info = _Info()
    x = np.zeros(op.n)
    rho = np.zeros(k_max)
    pres = np.zeros(k_max)
    alpha = np.zeros(k_max + 1)
    t = np.zeros(k_max + 2)
    u = np.zeros(k_max)
    dimq = op.m if mode == MODE_AB else op.n
    dims = op.n if mode == MODE_BA else op.m
    Q = np.zeros((k_max + 1, dimq)) if want_bases else None
    S = np.zeros((k_max + 1, dims)) if want_bases else None
    rc = lib().or_gkb(ctypes.byref(op.g), mode, _ptr(b), ctypes.byref(o), _ptr(x), _ptr(rho), _ptr(pres),
                      _ptr(alpha), _ptr(t), _ptr(Q), _ptr(S), _ptr(u), ctypes.byref(info))
    if rc != 0:
        raise ValueError("oracle gkb: invalid arguments")
    k = info.k_stop
    return GKBResult(x=x.reshape(op.image_shape), k_stop=k, reason=info.reason, residual=info.residual,
                     proj_residual=info.proj_residual, t1=info.t1, alpha1=info.alpha1, rho=rho[:k], pres=pres[:k],
                     alpha=alpha, t=t, Q=Q, S=S, u=u[:k], rre=None if xt is None else rre[:k])


@dataclass
class GMRESResult:
    x: np.ndarray
    k_stop: int
    reason: int
    residual: float
    proj_residual: float
    beta: float                      # ||r_0||
    rho: np.ndarray                  # ||A x_k - b||, k = 1..k_stop
    pres: np.ndarray                 # ||H_k u_k - beta e_1||
    H: Optional[np.ndarray] = None   # (k_stop + 1) x k_stop Hessenberg
    Q: Optional[np.ndarray] = None   # (k_stop + 1) x dimq Arnoldi basis (rows)
    rre: Optional[np.ndarray] = None


def gmres(op: Operator, mode: int, b, k_max: int, use_dp: bool = False, tau: float = 1.0,
          noise_norm: float = 0.0, rns_eps: float = 0.0, want_bases: bool = False, x_true=None) -> GMRESResult:
    """AB-GMRES (mode 0) or BA-GMRES (mode 1) from x_0 = 0 (Algs. "AB-GMRES",
    "BA-GMRES"; Arnoldi with modified Gram-Schmidt, eq. (proj) by the SVD of
    H_k).  Stops by the discrepancy principle, residual norm stagnation,
    breakdown or k_max, on the literal ||A x_k - b||."""
    if mode not in (MODE_AB, MODE_BA):
        raise ValueError("GMRES modes are MODE_AB and MODE_BA")
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    assert b.size == op.m
    xt = None if x_true is None else np.ascontiguousarray(np.asarray(x_true, dtype=np.float64).reshape(-1))
    rre = np.zeros(k_max)
    o = _Opts(k_max, 0.0, 1 if use_dp else 0, tau, noise_norm, 1, rns_eps,
              None if xt is None else xt.ctypes.data, None if xt is None else rre.ctypes.data)
    info = _Info()
    x = np.zeros(op.n)
    rho = np.zeros(k_max)
    pres = np.zeros(k_max)
    dimq = op.m if mode == MODE_AB else op.n
    H = np.zeros((k_max + 1, k_max)) if want_bases else None
    Q = np.zeros((k_max + 1, dimq)) if want_bases else None
    rc = lib().or_gmres(ctypes.byref(op.g), mode, _ptr(b), ctypes.byref(o), _ptr(x), _ptr(rho), _ptr(pres),
                        _ptr(H), _ptr(Q), ctypes.byref(info))
    if rc != 0:
        raise ValueError("oracle gmres: invalid arguments")
    k = info.k_stop
    return GMRESResult(x=x.reshape(op.image_shape), k_stop=k, reason=info.reason, residual=info.residual,
                       proj_residual=info.proj_residual, beta=info.t1, rho=rho[:k], pres=pres[:k],
                       H=None if H is None else H[:k + 1, :k], Q=None if Q is None else Q[:k + 1],
                       rre=None if xt is None else rre[:k])


def proj_solve(alpha, t, k: int, lam: float = 0.0):
    """u_k of eq. (proj GKB) with Tikhonov lam via the Jacobi SVD.  Returns
    (u, ||C_k u - t1 e1||, singular values)."""
    a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    tt = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    u = np.zeros(k)
    pr = np.zeros(1)
    sig = np.zeros(k)
    lib().or_proj_solve(k, _ptr(a), _ptr(tt), lam, _ptr(u), _ptr(pr), _ptr(sig))
    return u, float(pr[0]), sig


def jacobi_svd(Mat: np.ndarray):
    W = np.ascontiguousarray(np.array(Mat, dtype=np.float64))
    rows, cols = W.shape
    sig = np.zeros(cols)
    V = np.zeros((cols, cols))
    lib().or_jacobi_svd(rows, cols, _ptr(W), _ptr(sig), _ptr(V))
    return W, sig, V


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))
