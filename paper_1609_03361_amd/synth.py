"""Seeded synthetic inputs for the damped acoustic propagator.

This module only *makes inputs*: velocity/slowness models, damping sponges,
Ricker wavelets and source/receiver geometry.  It contains none of the
finite-difference method's arithmetic (no stencil, no time stepping, no
interpolation), so the CPU oracle and the HIP path can both be fed from it
without sharing any of the method.

Conventions (shared by every consumer):
  * arrays are C-contiguous with the depth axis z last (fastest):
    2D ``[nx][nz]``, 3D ``[nx][ny][nz]``;
  * coordinates are metres measured from grid index 0, FP64, ``[npts][ndim]``;
  * ``m`` is the squared slowness 1/v**2 (s^2/m^2) and ``eta`` the damping
    field (s/m^2), both FP32 (the wave equation of the seismic-inversion
    example, Section "Seismic Inversion Example");
  * wavelets and traces are time-major ``[nt][npts]`` FP32.

Workloads follow the paper's performance test (Section "Performance" of the
seismic example: layered model, absorbing sponge of 40 points per side,
10 Hz Ricker source) scaled to the sizes measured here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = [
    "ricker", "layered", "sponge", "cfl_dt", "line_receivers", "plane_receivers",
    "Problem", "config_2d_small", "config_3d_o8", "config_3d_o16",
    "config_batched_2d", "config_gradient_3d", "random_problem",
]


def ricker(f0: float, nt: int, dt: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet of peak frequency ``f0`` sampled at t_n = n*dt (FP64 → FP32).

    q(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2), t0 = 1/f0,
    amplitude 1.
    """
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def layered(shape, seed: int, vmin: float = 1500.0, vmax: float = 4500.0,
            nlayers: int = 6, perturb: float = 0.05, smooth: float = 3.0):
    """Seeded layered velocity model with a smoothed random perturbation.

    ``nlayers`` constant-velocity layers (velocities ``linspace(vmin, vmax)``
    increasing with depth) separated by ``nlayers-1`` random interface depths,
    times ``(1 + p)`` where ``p`` is Gaussian-smoothed white noise scaled to
    ``max|p| = perturb``.  Returns ``(m, v)``: FP32 squared slowness and the
    FP64 velocity it was rounded from.
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    nz = shape[-1]
    depths = np.sort(rng.uniform(0.05, 0.95, nlayers - 1)) * nz
    iface = np.round(depths).astype(np.int64)
    for k in range(1, len(iface)):            # make the interfaces distinct
        if iface[k] <= iface[k - 1]:
            iface[k] = iface[k - 1] + 1
    iface = np.clip(iface, 1, nz - 1)
    vel = np.linspace(vmin, vmax, nlayers)
    zidx = np.arange(nz)
    layer = np.searchsorted(iface, zidx, side="right")
    vz = vel[layer]                                     # [nz]
    p = gaussian_filter(rng.standard_normal(shape), sigma=smooth)
    p *= perturb / np.max(np.abs(p))
    v = vz.reshape((1,) * (len(shape) - 1) + (nz,)) * (1.0 + p)
    m = (1.0 / (v * v)).astype(np.float32)
    return m, v


def sponge(m: np.ndarray, h: float, width: int, vmax: float,
           reflection: float = 1e-3, free_top: bool = True) -> np.ndarray:
    """Absorbing sponge: eta = m * sigma with sigma = sigma_max (d/W)^2.

    ``d`` is the depth (in points) into the ``width``-point layer along each
    face; every face is damped except z = 0 when ``free_top``.  The corner
    value is the largest of the per-face values.  sigma_max =
    3 vmax ln(1/R) / (2 W h).
    """
    shape = m.shape
    ndim = len(shape)
    smax = 3.0 * vmax * math.log(1.0 / reflection) / (2.0 * width * h)
    prof = np.zeros(shape, dtype=np.float64)
    for a in range(ndim):
        n = shape[a]
        i = np.arange(n, dtype=np.float64)
        lo = np.clip(width - i, 0, None)                # depth into the low face
        hi = np.clip(i - (n - 1 - width), 0, None)      # depth into the high face
        if a == ndim - 1 and free_top:
            lo = np.zeros_like(lo)
        d = np.maximum(lo, hi) / width
        prof = np.maximum(prof, (d * d).reshape([n if b == a else 1 for b in range(ndim)]))
    return (m.astype(np.float64) * smax * prof).astype(np.float32)


def cfl_dt(h: float, vmax: float, cfl: float = 0.4) -> float:
    """Time step from a Courant number: dt = cfl * h / vmax."""
    return cfl * h / vmax


def line_receivers(n: int, x_max: float, z: float) -> np.ndarray:
    """2D receivers ``[n][2]`` along x = linspace(0, x_max) at depth z."""
    c = np.zeros((n, 2))
    c[:, 0] = np.linspace(0.0, x_max, n)
    c[:, 1] = z
    return c


def plane_receivers(n: int, x_max: float, y_max: float, z: float) -> np.ndarray:
    """3D receivers ``[n*n][3]`` on a linspace(0, max) x linspace(0, max) grid at depth z."""
    xs = np.linspace(0.0, x_max, n)
    ys = np.linspace(0.0, y_max, n)
    gx, gy = np.meshgrid(xs, ys, indexing="ij")
    c = np.zeros((n * n, 3))
    c[:, 0] = gx.ravel()
    c[:, 1] = gy.ravel()
    c[:, 2] = z
    return c


@dataclass
class Problem:
    """One single-shot problem: grid, coefficient fields, sources and receivers."""
    name: str
    shape: tuple
    spacing: tuple
    order: int
    dt: float
    nt: int
    m: np.ndarray                # FP32 [shape]
    eta: np.ndarray | None       # FP32 [shape] or None (no damping)
    src: np.ndarray              # FP64 [nsrc][ndim]
    q: np.ndarray                # FP32 [nt][nsrc]
    rec: np.ndarray              # FP64 [nrec][ndim]
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))


def config_2d_small(nt: int = 250) -> Problem:
    """2D, 101 x 101, h = 10 m, v = 1.5 km/s, order 4, CFL 0.4, no damping;
    10 Hz Ricker at the centre node, 101 receivers at depth index 2."""
    n, h, v = 101, 10.0, 1500.0
    m = np.full((n, n), 1.0 / (v * v), dtype=np.float32)
    dt = cfl_dt(h, v)
    src = np.array([[500.0, 500.0]])
    q = ricker(10.0, nt, dt).reshape(nt, 1)
    rec = line_receivers(101, 1000.0, 20.0)
    return Problem("2d-101-o4", (n, n), (h, h), 4, dt, nt, m, None, src, q, rec)


def _vmax(*ms) -> float:
    return max(float(np.max(1.0 / np.sqrt(mm.astype(np.float64)))) for mm in ms)


def config_3d_o8(n: int = 256, nt: int = 1000, seed: int = 2, nrec_side: int = 128,
                 order: int = 8, width: int = 40, f0: float = 15.0) -> Problem:
    """3D n^3 (default 256^3), h = 10 m, layered model, 40-point sponge,
    order 8, 15 Hz Ricker near the surface, nrec_side^2 receivers at depth index 2."""
    h = 10.0
    m, _ = layered((n, n, n), seed)
    vmax = _vmax(m)
    eta = sponge(m, h, min(width, n // 4), vmax)
    dt = cfl_dt(h, vmax)
    c = (n - 1) * h / 2.0
    src = np.array([[c, c, 25.0]])
    q = ricker(f0, nt, dt).reshape(nt, 1)
    rec = plane_receivers(nrec_side, (n - 1) * h, (n - 1) * h, 20.0)
    return Problem(f"3d-{n}-o{order}", (n, n, n), (h, h, h), order, dt, nt, m, eta, src, q, rec)


def config_3d_o16(n: int = 512, nt: int = 2000) -> Problem:
    """3D 512^3, order 16, same generator (seed 3), 256 x 256 receivers."""
    p = config_3d_o8(n=n, nt=nt, seed=3, nrec_side=256, order=16)
    p.name = f"3d-{n}-o16"
    return p


def config_batched_2d(nshots: int = 48, nx: int = 2001, nz: int = 801, nt: int = 2000,
                      order: int = 8, wmin: int = 400, nrec: int = 400, seed: int = 4):
    """Batched 2D shots on sub-apertures of one seeded ``nx x nz`` layered model.

    Shot s draws (from ``default_rng(1000*seed + s)``) a width w_s uniform in
    [wmin, nx] and an offset x0_s uniform in [0, nx - w_s]; its grid is the
    model columns [x0_s, x0_s + w_s) with its own 40-point sponge (left,
    right, bottom).  One 10 Hz Ricker at the window centre, 25 m deep, and
    ``nrec`` receivers across the window at 20 m.  All shots share dt.
    """
    h = 10.0
    m_full, _ = layered((nx, nz), seed)
    vmax = _vmax(m_full)
    dt = cfl_dt(h, vmax)
    q = ricker(10.0, nt, dt).reshape(nt, 1)
    shots = []
    for s in range(nshots):
        rng = np.random.default_rng(1000 * seed + s)
        w = int(rng.integers(wmin, nx, endpoint=True))
        x0 = int(rng.integers(0, nx - w, endpoint=True))
        m = np.ascontiguousarray(m_full[x0:x0 + w])
        eta = sponge(m, h, 40, vmax)
        src = np.array([[(w - 1) * h / 2.0, 25.0]])
        rec = line_receivers(nrec, (w - 1) * h, 20.0)
        shots.append(Problem(f"shot{s}-w{w}", (w, nz), (h, h), order, dt, nt, m, eta, src,
                             q.copy(), rec, extra={"x0": x0}))
    return shots


def config_gradient_3d(n: int = 200, nt: int = 1500, width: int = 40, nrec_side: int = 100,
                       seed: int = 5, order: int = 8):
    """FWI gradient problem: smooth layered m0 and a 'true' model with a +5 %
    Gaussian velocity anomaly at the centre; 4 shots at (x, y) in
    {0.25, 0.75}^2 of the extent, 25 m deep; nrec_side^2 receivers at 20 m.

    Returns ``(m0, m_true, eta, shots)`` where each shot is a Problem built
    on m0 (the observed data must be modelled on m_true by the caller).
    """
    h = 10.0
    shape = (n, n, n)
    m0, v0 = layered(shape, seed)
    L = (n - 1) * h
    ax = np.arange(n) * h
    gx, gy, gz = np.meshgrid(ax, ax, ax, indexing="ij", sparse=True)
    c = L / 2.0
    r2 = (gx - c) ** 2 + (gy - c) ** 2 + (gz - c) ** 2
    v_true = v0 * (1.0 + 0.05 * np.exp(-r2 / (2.0 * (0.1 * L) ** 2)))
    m_true = (1.0 / (v_true * v_true)).astype(np.float32)
    vmax = _vmax(m0, m_true)
    eta = sponge(m0, h, width, vmax)
    dt = cfl_dt(h, vmax)
    q = ricker(10.0, nt, dt).reshape(nt, 1)
    rec = plane_receivers(nrec_side, L, L, 20.0)
    shots = []
    for fx in (0.25, 0.75):
        for fy in (0.25, 0.75):
            src = np.array([[fx * L, fy * L, 25.0]])
            shots.append(Problem(f"grad-{n}-s{len(shots)}", shape, (h, h, h), order, dt, nt,
                                 m0, eta, src, q.copy(), rec))
    return m0, m_true, eta, shots


def random_problem(shape, order: int, nt: int, seed: int, nsrc: int = 3, nrec: int = 7,
                   damping: bool = True, cfl: float = 0.4, spacing=None) -> Problem:
    """Small randomized problem for parity sweeps: random smooth m, random
    sponge-free damping, random off-grid sources and receivers (some on the
    upper edges and some sharing cells), random wavelets."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    if spacing is None:
        spacing = tuple(float(x) for x in rng.uniform(8.0, 12.0, ndim))
    v = 1500.0 + 1500.0 * gaussian_filter(rng.uniform(0, 1, shape), 1.5)
    m = (1.0 / (v * v)).astype(np.float32)
    vmax = float(np.max(1.0 / np.sqrt(m.astype(np.float64))))
    eta = None
    if damping:
        eta = (m.astype(np.float64) * rng.uniform(0.0, 60.0, shape)).astype(np.float32)
    dt = cfl * min(spacing) / vmax
    ext = np.array([(s - 1) * hh for s, hh in zip(shape, spacing)])

    def pts(k):
        c = rng.uniform(0, 1, (k, ndim)) * ext
        if k >= 2:
            c[0] = ext                      # upper corner: exercises the edge clamp
            c[1] = 0.0                      # lower corner
        if k >= 4:
            c[3] = c[2]                     # two points on the same spot
        return c

    src = pts(nsrc)
    rec = pts(nrec)
    q = rng.standard_normal((nt, nsrc)).astype(np.float32)
    return Problem(f"rand-{shape}-o{order}-s{seed}", shape, tuple(spacing), order, dt, nt,
                   m, eta, src, q, rec)
