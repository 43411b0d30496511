"""CPU oracle for the damped acoustic propagator — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It never imports the product package and shares no code
with the HIP library: it is a ctypes wrapper around ``wave_oracle.c`` (plain
loops, FP64) plus ``numpy_ref`` (an independent NumPy re-statement for tiny
grids).

Every function takes plain arrays: shape, spacing, order, dt, nt, FP32 model
fields (upcast exactly to FP64), FP64 coordinates in metres, FP32 wavelets.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import lib_path, build as _build

__all__ = ["fd_weights", "sparse_weights", "laplacian", "forward", "adjoint", "gradient",
           "diffusion", "num_threads", "OracleError"]

_LIBS: dict = {}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("shape", C.c_int64 * 3), ("spacing", C.c_double * 3),
                ("order", C.c_int32), ("dt", C.c_double), ("nt", C.c_int32)]


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


def _lib(precision: str = "f64"):
    if precision not in _LIBS:
        path = lib_path(precision)
        if not os.path.exists(path):
            _build()
        lib = C.CDLL(path)
        lib.oracle_fd_weights.argtypes = [C.c_int, _D]
        lib.oracle_sparse_weights.argtypes = [C.POINTER(_Grid), C.c_int, _D, _I64, _D]
        lib.oracle_laplacian.argtypes = [C.POINTER(_Grid), _D, _D]
        lib.oracle_forward.argtypes = [C.POINTER(_Grid), _D, _D, C.c_int, _D, _D, C.c_int, _D, _D,
                                       _D, _D, C.c_int, _D, _D, _D, _D, _D]
        lib.oracle_adjoint.argtypes = [C.POINTER(_Grid), _D, _D, C.c_int, _D, _D, C.c_int, _D, _D,
                                       _D, _D]
        lib.oracle_gradient.argtypes = [C.POINTER(_Grid), _D, _D, C.c_int, _D, _D, C.c_int, _D,
                                        _D, _D, _D, _D, _D]
        lib.oracle_diffusion.argtypes = [C.POINTER(_Grid), _D, _D, _D]
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_real_bytes.restype = C.c_int
        _LIBS[precision] = lib
    return _LIBS[precision]


def num_threads() -> int:
    """OpenMP threads the oracle's grid loop uses (OMP_NUM_THREADS or all cores)."""
    return int(_lib().oracle_num_threads())


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a, n=None):
    if a is None:
        return None
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and out.size != n:
        raise ValueError(f"expected {n} values, got {out.size}")
    return out


def _grid(shape, spacing, order, dt=1.0, nt=0) -> _Grid:
    g = _Grid()
    g.ndim = len(shape)
    for a in range(3):
        g.shape[a] = int(shape[a]) if a < len(shape) else 0
        g.spacing[a] = float(spacing[a]) if a < len(shape) else 0.0
    g.order = int(order)
    g.dt = float(dt)
    g.nt = int(nt)
    return g


def fd_weights(order: int) -> np.ndarray:
    """c_0..c_k of the order-2k central second derivative (unit spacing)."""
    c = np.zeros(9)
    rc = _lib().oracle_fd_weights(int(order), _p(c))
    if rc:
        raise OracleError(rc, "fd_weights")
    return c[: order // 2 + 1].copy()


def sparse_weights(shape, spacing, coords):
    """Multilinear corner indices ``[npts][2^d]`` (flat, C order) and weights."""
    coords = _f64(coords).reshape(-1, len(shape))
    n = coords.shape[0]
    nc = 1 << len(shape)
    corner = np.zeros((n, nc), dtype=np.int64)
    w = np.zeros((n, nc))
    rc = _lib().oracle_sparse_weights(C.byref(_grid(shape, spacing, 2)), n, _p(coords),
                                      corner.ctypes.data_as(_I64), _p(w))
    if rc:
        raise OracleError(rc, "sparse_weights")
    return corner, w


def laplacian(shape, spacing, order, u, precision="f64") -> np.ndarray:
    """L u with the zero extension outside the grid."""
    u = _f64(u).reshape(shape)
    out = np.zeros(shape)
    rc = _lib(precision).oracle_laplacian(C.byref(_grid(shape, spacing, order)), _p(u), _p(out))
    if rc:
        raise OracleError(rc, "laplacian")
    return out


def forward(shape, spacing, order, dt, nt, m, eta=None, src=None, q=None, rec=None,
            u_prev0=None, u0=None, force_pat=None, force_t=None, want_final=True,
            want_hist=False, precision="f64"):
    """Forward modelling; returns dict with ``d`` [nt][nrec], ``u`` = u^nt,
    ``u_prev`` = u^{nt-1}, and ``hist`` [nt+2][shape] (u^{-1}..u^nt) if asked."""
    ndim = len(shape)
    N = int(np.prod(shape))
    m = _f64(m, N)
    eta = _f64(eta, N)
    src = np.zeros((0, ndim)) if src is None else _f64(src).reshape(-1, ndim)
    rec = np.zeros((0, ndim)) if rec is None else _f64(rec).reshape(-1, ndim)
    ns, nr = src.shape[0], rec.shape[0]
    q = _f64(q, nt * ns) if ns else None
    d = np.zeros((nt, nr)) if nr else None
    nforce = 0
    if force_pat is not None:
        force_pat = _f64(force_pat).reshape(-1, N)
        nforce = force_pat.shape[0]
        force_t = _f64(force_t, nt * nforce)
    uf = np.zeros(shape) if want_final else None
    upf = np.zeros(shape) if want_final else None
    hist = np.zeros((nt + 2,) + tuple(shape)) if want_hist else None
    rc = _lib(precision).oracle_forward(
        C.byref(_grid(shape, spacing, order, dt, nt)), _p(m), _p(eta), ns, _p(src), _p(q),
        nr, _p(rec), _p(d), _p(_f64(u_prev0, N)), _p(_f64(u0, N)), nforce, _p(force_pat),
        _p(force_t), _p(uf), _p(upf), _p(hist))
    if rc:
        raise OracleError(rc, "forward")
    return {"d": d if nr else np.zeros((nt, 0)), "u": uf, "u_prev": upf, "hist": hist}


def adjoint(shape, spacing, order, dt, nt, m, eta, rec, dres, src, want_hist=False,
            precision="f64"):
    """Adjoint modelling driven by receiver data ``dres`` [nt][nrec]; returns
    dict with ``qadj`` [nt][nsrc], ``v`` = v^0 and optional ``hist`` v^0..v^nt."""
    ndim = len(shape)
    N = int(np.prod(shape))
    rec = _f64(rec).reshape(-1, ndim)
    src = _f64(src).reshape(-1, ndim)
    nr, ns = rec.shape[0], src.shape[0]
    dres = _f64(dres, nt * nr)
    qadj = np.zeros((nt, ns))
    v = np.zeros(shape)
    hist = np.zeros((nt + 1,) + tuple(shape)) if want_hist else None
    rc = _lib(precision).oracle_adjoint(
        C.byref(_grid(shape, spacing, order, dt, nt)), _p(_f64(m, N)), _p(_f64(eta, N)), nr,
        _p(rec), _p(dres), ns, _p(src), _p(qadj), _p(v), _p(hist))
    if rc:
        raise OracleError(rc, "adjoint")
    return {"qadj": qadj, "v": v, "hist": hist}


def gradient(shape, spacing, order, dt, nt, m, eta, src, q, rec, d_obs, sbp=False,
             precision="f64"):
    """Misfit J and its gradient with respect to m for one shot (full storage)."""
    ndim = len(shape)
    N = int(np.prod(shape))
    src = _f64(src).reshape(-1, ndim)
    rec = _f64(rec).reshape(-1, ndim)
    ns, nr = src.shape[0], rec.shape[0]
    g = np.zeros(shape)
    gs = np.zeros(shape) if sbp else None
    J = np.zeros(1)
    dsyn = np.zeros((nt, nr))
    rc = _lib(precision).oracle_gradient(
        C.byref(_grid(shape, spacing, order, dt, nt)), _p(_f64(m, N)), _p(_f64(eta, N)), ns,
        _p(src), _p(_f64(q, nt * ns)), nr, _p(rec), _p(_f64(d_obs, nt * nr)), _p(g), _p(gs),
        _p(J), _p(dsyn))
    if rc:
        raise OracleError(rc, "gradient")
    return {"grad": g, "grad_sbp": gs, "J": float(J[0]), "d": dsyn}


def diffusion(shape, spacing, order, dt, nt, a, u0, precision="f64"):
    """Forward-Euler diffusion u^{n+1} = u^n + dt a L u^n from u0; returns u^nt."""
    N = int(np.prod(shape))
    out = np.zeros(shape)
    rc = _lib(precision).oracle_diffusion(C.byref(_grid(shape, spacing, order, dt, nt)),
                                          _p(_f64(a, N)), _p(_f64(u0, N)), _p(out))
    if rc:
        raise OracleError(rc, "diffusion")
    return out
