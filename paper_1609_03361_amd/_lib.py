"""ctypes view of the C ABI in include/wave.h (argument marshalling only).

The shared library is built in-tree (``paper_1609_03361_amd/_build/libwave.so``)
by ``build.py``; loading fails loudly if it is missing — there is no other
implementation behind these names.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libwave.so")

WAVE_OK, WAVE_EINVAL, WAVE_ECFL, WAVE_ERANGE, WAVE_EWORKSPACE, WAVE_EHIP = 0, -1, -2, -3, -4, -5
WAVE_OP_FORWARD, WAVE_OP_ADJOINT, WAVE_OP_GRADIENT, WAVE_OP_FORWARD_CKPT, WAVE_OP_BACKWARD = \
    0, 1, 2, 3, 4
WAVE_MISFIT_WORKSPACE_BYTES = 4096
WAVE_NOALLOC_WORKSPACE_BYTES = 64 << 20
CKPT_DTYPES = {"fp32": 0, "bf16": 1, "fp16": 2}
_NAMES = {0: "WAVE_OK", -1: "WAVE_EINVAL", -2: "WAVE_ECFL", -3: "WAVE_ERANGE",
          -4: "WAVE_EWORKSPACE", -5: "WAVE_EHIP"}

EXPORTS = ["wave_workspace_size", "wave_checkpoint_size", "wave_forward", "wave_adjoint",
           "wave_backward", "wave_gradient", "wave_batch_workspace_size", "wave_forward_batch",
           "wave_tune", "wave_tune_batch", "wave_tune_shot", "wave_last_batch_mode", "wave_diffusion",
           "wave_set_profiling", "wave_last_loop", "wave_misfit", "wave_release",
           "wave_tile_candidates", "wave_resolve_tile", "wave_forward_noalloc",
           "wave_last_error", "wave_version"]
WAVE_FLAG_NO_GRAPH = 1
WAVE_FLAG_PERSISTENT = 2
WAVE_FLAG_TUNE_IMAGING = 4


class WaveError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("space_order", C.c_int32), ("shape", C.c_int64 * 3),
                ("spacing", C.c_double * 3), ("dt", C.c_double), ("nt", C.c_int32),
                ("reserved", C.c_int32)]


class Points(C.Structure):
    _fields_ = [("npts", C.c_int32), ("reserved", C.c_int32), ("coords", C.POINTER(C.c_double))]


class Opts(C.Structure):
    _fields_ = [("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("ckpt_every", C.c_int32), ("ckpt_dtype", C.c_int32), ("tile", C.c_int32),
                ("flags", C.c_int32)]


class Shot(C.Structure):
    _fields_ = [("grid", Grid), ("m", C.c_void_p), ("eta", C.c_void_p), ("src", Points),
                ("q", C.c_void_p), ("rec", Points), ("d", C.c_void_p), ("u_final", C.c_void_p)]


_lib = None


def lib():
    """Load libwave.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, VP, I32 = C.POINTER, C.c_void_p, C.c_int32
        L.wave_workspace_size.argtypes = [I32, P(Grid), P(Points), P(Points), P(Opts),
                                          P(C.c_size_t)]
        L.wave_checkpoint_size.argtypes = [P(Grid), P(Opts), P(C.c_size_t)]
        L.wave_forward.argtypes = [P(Grid), VP, VP, P(Points), VP, P(Points), VP, VP, VP, P(Opts), VP]
        L.wave_adjoint.argtypes = [P(Grid), VP, VP, P(Points), VP, P(Points), VP, VP, P(Opts), VP]
        L.wave_backward.argtypes = [P(Grid), VP, VP, P(Points), VP, P(Points), VP, VP, VP, VP,
                                    P(Opts), VP]
        L.wave_gradient.argtypes = [P(Grid), VP, VP, P(Points), VP, P(Points), VP, VP, VP, VP,
                                    P(Opts), VP]
        L.wave_batch_workspace_size.argtypes = [I32, P(Shot), P(Opts), P(C.c_size_t)]
        L.wave_forward_batch.argtypes = [I32, P(Shot), P(Opts), VP]
        L.wave_tune.argtypes = [P(Grid), P(Opts), I32, VP, P(C.c_int32), P(C.c_double)]
        L.wave_tune_batch.argtypes = [I32, P(Shot), P(Opts), I32, VP, P(C.c_int32), P(C.c_double)]
        L.wave_tune_shot.argtypes = [P(Grid), VP, VP, P(Points), P(Points), P(Opts), I32, VP,
                                     P(C.c_int32), P(C.c_double)]
        for name in ("wave_workspace_size", "wave_checkpoint_size", "wave_forward", "wave_adjoint",
                     "wave_backward", "wave_gradient", "wave_batch_workspace_size",
                     "wave_forward_batch", "wave_tune", "wave_tune_batch", "wave_tune_shot"):
            getattr(L, name).restype = C.c_int
        L.wave_set_profiling.argtypes = [I32]
        L.wave_set_profiling.restype = C.c_int
        L.wave_last_loop.argtypes = [P(C.c_double), P(C.c_int64)]
        L.wave_last_loop.restype = C.c_int
        L.wave_last_batch_mode.restype = C.c_int
        L.wave_diffusion.argtypes = [P(Grid), VP, VP, VP, P(Opts), VP]
        L.wave_diffusion.restype = C.c_int
        L.wave_misfit.argtypes = [VP, VP, C.c_int64, VP, VP, P(Opts), VP]
        L.wave_misfit.restype = C.c_int
        L.wave_tile_candidates.argtypes = [P(Grid), P(C.c_int32), I32, P(C.c_int32)]
        L.wave_tile_candidates.restype = C.c_int
        L.wave_resolve_tile.argtypes = [P(Grid), I32, P(C.c_int32)]
        L.wave_resolve_tile.restype = C.c_int
        L.wave_forward_noalloc.argtypes = [P(Grid), VP, VP, P(Points), VP, P(Points), VP, VP, VP]
        L.wave_forward_noalloc.restype = C.c_int
        L.wave_release.argtypes = []
        L.wave_release.restype = C.c_int
        L.wave_last_error.restype = C.c_char_p
        L.wave_version.restype = C.c_char_p
        _lib = L
        # release the library's per-thread HIP objects (graph, capture stream,
        # events, pinned staging) before the runtime itself shuts down
        atexit.register(release)
    return _lib


def release() -> None:
    """Destroy what libwave.so keeps for the calling thread (see wave_release)."""
    if _lib is not None:
        _lib.wave_release()


def check(rc: int, where: str) -> None:
    if rc != WAVE_OK:
        raise WaveError(rc, where, lib().wave_last_error().decode())


def make_grid(shape, spacing, order, dt, nt) -> Grid:
    g = Grid()
    g.ndim = len(shape)
    for a in range(3):
        g.shape[a] = int(shape[a]) if a < len(shape) else 0
        g.spacing[a] = float(spacing[a]) if a < len(shape) else 0.0
    g.space_order = int(order)
    g.dt = float(dt)
    g.nt = int(nt)
    g.reserved = 0
    return g


class HostPoints:
    """Keeps the FP64 coordinate array alive while a call uses it."""

    def __init__(self, coords, ndim: int):
        if coords is None:
            self.arr = np.zeros((0, ndim))
        else:
            self.arr = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).reshape(-1, ndim))
        self.s = Points()
        self.s.npts = self.arr.shape[0]
        self.s.reserved = 0
        self.s.coords = self.arr.ctypes.data_as(C.POINTER(C.c_double)) if self.arr.size else None

    @property
    def npts(self) -> int:
        return self.arr.shape[0]


def make_opts(workspace_ptr=0, workspace_bytes=0, ckpt_every=0, ckpt_dtype="fp32", tile=0,
              flags=0) -> Opts:
    o = Opts()
    o.workspace = workspace_ptr or None
    o.workspace_bytes = int(workspace_bytes)
    o.ckpt_every = int(ckpt_every)
    o.ckpt_dtype = CKPT_DTYPES[ckpt_dtype] if isinstance(ckpt_dtype, str) else int(ckpt_dtype)
    o.tile = int(tile)
    o.flags = int(flags)
    return o


def set_profiling(on: bool) -> None:
    check(lib().wave_set_profiling(1 if on else 0), "wave_set_profiling")


def last_loop():
    """(milliseconds, step launches) of the last profiled call on this thread."""
    ms = C.c_double(0)
    n = C.c_int64(0)
    check(lib().wave_last_loop(C.byref(ms), C.byref(n)), "wave_last_loop")
    return ms.value, n.value
