"""PyTorch-facing wrappers over the C ABI (device memory and streams only).

Every step of the method runs inside libwave.so; these functions allocate
the caller-owned buffers (outputs, workspace, checkpoints) as torch tensors
and pass raw pointers plus the current HIP stream.

Arguments mirror the paper's problem statement forward(model, nt, dt, h,
order): ``m`` and ``eta`` are FP32 device tensors of the grid's shape (z
fastest), ``spacing`` the grid spacing per axis in metres, ``src``/``rec``
host FP64 coordinates ``[n][ndim]`` in metres, ``q`` the source wavelets
``[nt][nsrc]`` (FP32, device).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

__all__ = ["Geometry", "forward", "adjoint", "backward", "gradient", "checkpoint_bytes",
           "forward_batch", "tune", "tune_batch", "tile_candidates", "resolve_tile", "diffusion",
           "misfit", "WaveFn", "wave_apply"]


def _ptr(t):
    return None if t is None else t.data_ptr()


def _need(t, name, shape=None):
    if t is None:
        return
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _need_checkpoint(ck, geom, ckpt_every, ckpt_dtype):
    """The library cannot see the size of the checkpoint buffer: check it here."""
    if not (ck.is_cuda and ck.dtype == torch.uint8 and ck.is_contiguous()):
        raise ValueError("checkpoint must be a contiguous uint8 device tensor")
    need = checkpoint_bytes(geom, ckpt_every, ckpt_dtype)
    if ck.numel() < need:
        raise ValueError(f"checkpoint holds {ck.numel()} bytes; ckpt_every={ckpt_every}, "
                         f"ckpt_dtype={ckpt_dtype} need {need}")


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _workspace(op, grid, sp, rp, opts_kw, dev):
    nbytes = C.c_size_t(0)
    o = L.make_opts(**opts_kw)
    L.check(L.lib().wave_workspace_size(op, C.byref(grid), C.byref(sp.s), C.byref(rp.s),
                                        C.byref(o), C.byref(nbytes)), "wave_workspace_size")
    buf = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    base = buf.data_ptr()
    off = (-base) % 256
    o = L.make_opts(base + off, int(nbytes.value), **opts_kw)
    return buf, o


@dataclass
class Geometry:
    """Grid, time axis and sparse-point positions of one shot."""
    shape: tuple
    spacing: tuple
    order: int
    dt: float
    nt: int
    src: object = None     # host FP64 [nsrc][ndim]
    rec: object = None     # host FP64 [nrec][ndim]

    def grid(self):
        return L.make_grid(self.shape, self.spacing, self.order, self.dt, self.nt)

    def points(self):
        nd = len(self.shape)
        return L.HostPoints(self.src, nd), L.HostPoints(self.rec, nd)


def checkpoint_bytes(geom: Geometry, ckpt_every=0, ckpt_dtype="fp32") -> int:
    n = C.c_size_t(0)
    o = L.make_opts(ckpt_every=ckpt_every, ckpt_dtype=ckpt_dtype)
    L.check(L.lib().wave_checkpoint_size(C.byref(geom.grid()), C.byref(o), C.byref(n)),
            "wave_checkpoint_size")
    return int(n.value)


def forward(geom: Geometry, m, eta=None, q=None, return_final=False, checkpoint=None,
            ckpt_every=0, ckpt_dtype="fp32", tile=0):
    """Modelled traces d [nt][nrec] (and u^nt if ``return_final``).
    ``checkpoint``: optional uint8 device tensor of checkpoint_bytes() that
    receives the snapshots wave_backward replays."""
    _need(m, "m", geom.shape)
    _need(eta, "eta", geom.shape)
    sp, rp = geom.points()
    if sp.npts:
        _need(q, "q", (geom.nt, sp.npts))
    dev = m.device
    grid = geom.grid()
    kw = dict(ckpt_every=ckpt_every, ckpt_dtype=ckpt_dtype, tile=tile)
    op = L.WAVE_OP_FORWARD
    if checkpoint is not None:
        _need_checkpoint(checkpoint, geom, ckpt_every, ckpt_dtype)
        op = L.WAVE_OP_FORWARD_CKPT
    ws, o = _workspace(op, grid, sp, rp, kw, dev)
    d = torch.empty((geom.nt, rp.npts), dtype=torch.float32, device=dev)
    uf = torch.empty(geom.shape, dtype=torch.float32, device=dev) if return_final else None
    L.check(L.lib().wave_forward(C.byref(grid), _ptr(m), _ptr(eta), C.byref(sp.s), _ptr(q),
                                 C.byref(rp.s), _ptr(d) if rp.npts else None, _ptr(uf),
                                 _ptr(checkpoint), C.byref(o), _stream(dev)), "wave_forward")
    return (d, uf) if return_final else d


def adjoint(geom: Geometry, m, eta, d, return_final=False, tile=0):
    """Adjoint modelling: receiver data d [nt][nrec] -> q_adj [nt][nsrc] (and v^0)."""
    _need(m, "m", geom.shape)
    _need(eta, "eta", geom.shape)
    sp, rp = geom.points()
    _need(d, "d", (geom.nt, rp.npts))
    dev = m.device
    grid = geom.grid()
    ws, o = _workspace(L.WAVE_OP_ADJOINT, grid, sp, rp, dict(tile=tile), dev)
    qa = torch.empty((geom.nt, sp.npts), dtype=torch.float32, device=dev)
    vf = torch.empty(geom.shape, dtype=torch.float32, device=dev) if return_final else None
    L.check(L.lib().wave_adjoint(C.byref(grid), _ptr(m), _ptr(eta), C.byref(rp.s), _ptr(d),
                                 C.byref(sp.s), _ptr(qa) if sp.npts else None, _ptr(vf),
                                 C.byref(o), _stream(dev)), "wave_adjoint")
    return (qa, vf) if return_final else qa


def backward(geom: Geometry, m, eta, q, r, checkpoint, ckpt_every=0, ckpt_dtype="fp32",
             want_grad_q=True, tile=0):
    """dJ/dm (and dJ/dq) for the adjoint source r = dJ/dd, replaying ``checkpoint``."""
    _need(m, "m", geom.shape)
    _need(eta, "eta", geom.shape)
    sp, rp = geom.points()
    _need(r, "r", (geom.nt, rp.npts))
    _need_checkpoint(checkpoint, geom, ckpt_every, ckpt_dtype)
    dev = m.device
    grid = geom.grid()
    kw = dict(ckpt_every=ckpt_every, ckpt_dtype=ckpt_dtype, tile=tile)
    ws, o = _workspace(L.WAVE_OP_BACKWARD, grid, sp, rp, kw, dev)
    g = torch.empty(geom.shape, dtype=torch.float32, device=dev)
    gq = torch.empty((geom.nt, sp.npts), dtype=torch.float32, device=dev) \
        if (want_grad_q and sp.npts) else None
    L.check(L.lib().wave_backward(C.byref(grid), _ptr(m), _ptr(eta), C.byref(sp.s), _ptr(q),
                                  C.byref(rp.s), _ptr(r), _ptr(checkpoint), _ptr(g), _ptr(gq),
                                  C.byref(o), _stream(dev)), "wave_backward")
    return g, gq


def gradient(geom: Geometry, m, eta, q, d_obs, ckpt_every=0, ckpt_dtype="fp32",
             return_data=False, tile=0):
    """Misfit J = 1/2 ||d - d_obs||^2 (device scalar) and dJ/dm for one shot."""
    _need(m, "m", geom.shape)
    _need(eta, "eta", geom.shape)
    sp, rp = geom.points()
    _need(d_obs, "d_obs", (geom.nt, rp.npts))
    dev = m.device
    grid = geom.grid()
    kw = dict(ckpt_every=ckpt_every, ckpt_dtype=ckpt_dtype, tile=tile)
    ws, o = _workspace(L.WAVE_OP_GRADIENT, grid, sp, rp, kw, dev)
    g = torch.empty(geom.shape, dtype=torch.float32, device=dev)
    J = torch.empty((), dtype=torch.float32, device=dev)
    dsyn = torch.empty((geom.nt, rp.npts), dtype=torch.float32, device=dev) if return_data else None
    L.check(L.lib().wave_gradient(C.byref(grid), _ptr(m), _ptr(eta), C.byref(sp.s), _ptr(q),
                                  C.byref(rp.s), _ptr(d_obs), _ptr(g), _ptr(J), _ptr(dsyn),
                                  C.byref(o), _stream(dev)), "wave_gradient")
    return (J, g, dsyn) if return_data else (J, g)


def tile_id(variant: int, xchunk: int) -> int:
    """Public tile id of the streaming kernel: block-shape variant and x-chunk length."""
    return (int(variant) << 16) | int(xchunk)


def tile_candidates(geom: Geometry):
    """Tile ids the autotuner times on this grid (distinct launches)."""
    grid = geom.grid()
    n = C.c_int32(0)
    L.check(L.lib().wave_tile_candidates(C.byref(grid), None, 0, C.byref(n)), "wave_tile_candidates")
    ids = (C.c_int32 * max(n.value, 1))()
    L.check(L.lib().wave_tile_candidates(C.byref(grid), ids, n.value, C.byref(n)),
            "wave_tile_candidates")
    return [int(ids[i]) for i in range(n.value)]


def resolve_tile(geom: Geometry, tile: int = 0) -> int:
    """The tile id a step launch on this grid uses for the requested one."""
    grid = geom.grid()
    out = C.c_int32(0)
    L.check(L.lib().wave_resolve_tile(C.byref(grid), int(tile), C.byref(out)), "wave_resolve_tile")
    return int(out.value)


def tune(geom: Geometry, steps: int = 20, device=None, imaging=False, m=None, eta=None):
    """Time every candidate tile on this grid; returns (tile id, us per step).
    The winner is cached for later calls with tile=0; with ``imaging`` the
    adjoint step with the imaging condition is tuned (and cached) instead.
    Given the model ``m`` (and ``eta``), the step is timed as this shot runs
    it, with its sources and receivers injected and sampled (wave_tune_shot);
    otherwise on the bare grid (wave_tune)."""
    if m is not None:
        _need(m, "m", geom.shape)
        _need(eta, "eta", geom.shape)
        dev = m.device
        grid = geom.grid()
        sp, rp = geom.points()
        flags = L.WAVE_FLAG_TUNE_IMAGING if imaging else 0
        op = L.WAVE_OP_ADJOINT if imaging else L.WAVE_OP_FORWARD
        ws, o = _workspace(op, grid, sp, rp, dict(flags=flags), dev)
        t = C.c_int32(0)
        us = C.c_double(0)
        L.check(L.lib().wave_tune_shot(C.byref(grid), _ptr(m), _ptr(eta), C.byref(sp.s),
                                       C.byref(rp.s), C.byref(o), int(steps), _stream(dev),
                                       C.byref(t), C.byref(us)), "wave_tune_shot")
        return int(t.value), float(us.value)
    dev = torch.device(device or "cuda:0")
    grid = geom.grid()
    empty = L.HostPoints(None, len(geom.shape))
    flags = L.WAVE_FLAG_TUNE_IMAGING if imaging else 0
    ws, o = _workspace(L.WAVE_OP_FORWARD, grid, empty, empty, dict(flags=flags), dev)
    t = C.c_int32(0)
    us = C.c_double(0)
    L.check(L.lib().wave_tune(C.byref(grid), C.byref(o), int(steps), _stream(dev), C.byref(t),
                              C.byref(us)), "wave_tune")
    return int(t.value), float(us.value)


class _Batch:
    """Marshals a list of (geometry, m, eta, q) into wave_shot structs."""

    def __init__(self, shots, return_final):
        self.keep = []
        n = len(shots)
        self.arr = (L.Shot * n)()
        self.d, self.uf = [], []
        for i, (geom, m, eta, q) in enumerate(shots):
            _need(m, f"shot {i} m", geom.shape)
            _need(eta, f"shot {i} eta", geom.shape)
            sp, rp = geom.points()
            if sp.npts:
                _need(q, f"shot {i} q", (geom.nt, sp.npts))
            d = torch.empty((geom.nt, rp.npts), dtype=torch.float32, device=m.device)
            uf = torch.empty(geom.shape, dtype=torch.float32, device=m.device) if return_final else None
            s = self.arr[i]
            s.grid = geom.grid()
            s.m, s.eta, s.q = _ptr(m), _ptr(eta), _ptr(q)
            s.src, s.rec = sp.s, rp.s
            s.d = _ptr(d) if rp.npts else None
            s.u_final = _ptr(uf)
            self.keep += [sp, rp, m, eta, q]
            self.d.append(d)
            self.uf.append(uf)
        self.n = n
        self.dev = shots[0][1].device

    def workspace(self, **kw):
        nbytes = C.c_size_t(0)
        o = L.make_opts(**kw)
        L.check(L.lib().wave_batch_workspace_size(self.n, self.arr, C.byref(o), C.byref(nbytes)),
                "wave_batch_workspace_size")
        buf = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.dev)
        off = (-buf.data_ptr()) % 256
        return buf, L.make_opts(buf.data_ptr() + off, int(nbytes.value), **kw)


def forward_batch(shots, return_final=False, tile=0, graph=True, persistent=False):
    """Forward-model many shots: one launch per step over all shots, replayed
    from a hipGraph (``graph``), or one persistent launch for all steps
    (``persistent``).  ``shots``: list of (Geometry, m, eta, q).  Returns the
    list of traces (and of final wavefields if ``return_final``)."""
    B = _Batch(shots, return_final)
    flags = (0 if graph else L.WAVE_FLAG_NO_GRAPH) | (L.WAVE_FLAG_PERSISTENT if persistent else 0)
    ws, o = B.workspace(tile=tile, flags=flags)
    L.check(L.lib().wave_forward_batch(B.n, B.arr, C.byref(o), _stream(B.dev)),
            "wave_forward_batch")
    return (B.d, B.uf) if return_final else B.d


def last_batch_mode() -> int:
    """How the last forward_batch on this thread ran: 0 per-step launches
    replayed from a hipGraph, 1 per-step launches, 2 one persistent launch,
    3 one persistent launch replayed from a hipGraph."""
    return int(L.lib().wave_last_batch_mode())


def misfit(d, d_obs, return_residual=False):
    """J = 1/2 sum (d - d_obs)^2 as a device scalar (wave_misfit), and the
    residual r = d - d_obs if ``return_residual``."""
    _need(d, "d")
    _need(d_obs, "d_obs", tuple(d.shape))
    dev = d.device
    ws = torch.empty(L.WAVE_MISFIT_WORKSPACE_BYTES + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    o = L.make_opts(ws.data_ptr() + off, L.WAVE_MISFIT_WORKSPACE_BYTES)
    J = torch.empty((), dtype=torch.float32, device=dev)
    r = torch.empty_like(d) if return_residual else None
    L.check(L.lib().wave_misfit(_ptr(d), _ptr(d_obs), d.numel(), _ptr(r), _ptr(J), C.byref(o),
                                _stream(dev)), "wave_misfit")
    return (J, r) if return_residual else J


def tune_batch(shots, steps: int = 10):
    """Tile autotuner for a batch; returns (tile id, us per step)."""
    B = _Batch(shots, False)
    ws, o = B.workspace()
    t = C.c_int32(0)
    us = C.c_double(0)
    L.check(L.lib().wave_tune_batch(B.n, B.arr, C.byref(o), int(steps), _stream(B.dev),
                                    C.byref(t), C.byref(us)), "wave_tune_batch")
    return int(t.value), float(us.value)


def diffusion(shape, spacing, order, dt, nt, a, u0, tile=0):
    """Forward-Euler diffusion u^{n+1} = u^n + dt a L u^n (the paper's diffusion
    example) from u0 on the step kernel; returns u^nt."""
    _need(a, "a", shape)
    _need(u0, "u0", shape)
    dev = a.device
    grid = L.make_grid(shape, spacing, order, dt, nt)
    empty = L.HostPoints(None, len(shape))
    ws, o = _workspace(L.WAVE_OP_FORWARD, grid, empty, empty, dict(tile=tile), dev)
    out = torch.empty(tuple(shape), dtype=torch.float32, device=dev)
    L.check(L.lib().wave_diffusion(C.byref(grid), _ptr(a), _ptr(u0), _ptr(out), C.byref(o),
                                   _stream(dev)), "wave_diffusion")
    return out


class WaveFn(torch.autograd.Function):
    """d = F(m, q): forward modelling with checkpointed snapshots; the backward
    is the hand-written adjoint with the imaging condition (wave_backward)."""

    @staticmethod
    def forward(ctx, m, q, eta, geom, ckpt_every=0, ckpt_dtype="fp32"):
        ck = torch.empty(checkpoint_bytes(geom, ckpt_every, ckpt_dtype), dtype=torch.uint8,
                         device=m.device)
        d = forward(geom, m.detach(), None if eta is None else eta.detach(), q.detach(),
                    checkpoint=ck, ckpt_every=ckpt_every, ckpt_dtype=ckpt_dtype)
        ctx.save_for_backward(m, q, eta, ck)
        ctx.geom, ctx.ck_every, ctx.ck_dtype = geom, ckpt_every, ckpt_dtype
        return d

    @staticmethod
    def backward(ctx, grad_d):
        m, q, eta, ck = ctx.saved_tensors
        g, gq = backward(ctx.geom, m.detach(), None if eta is None else eta.detach(), q.detach(),
                         grad_d.detach().contiguous().float(), ck, ctx.ck_every, ctx.ck_dtype,
                         want_grad_q=ctx.needs_input_grad[1])
        return g, gq, None, None, None, None


def wave_apply(geom: Geometry, m, q, eta=None, ckpt_every=0, ckpt_dtype="fp32"):
    """Differentiable forward modelling: traces as a function of (m, q)."""
    return WaveFn.apply(m, q, eta, geom, ckpt_every, ckpt_dtype)
