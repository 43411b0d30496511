"""The oracle against continuum physics (section "Seismic Inversion Example",
equation eqn:acoustic): a point source in a homogeneous 2D medium without
damping, compared with the free-space Green's function before any boundary
reflection arrives.

For (1/c^2) u_tt - lap(u) = f, the 2D Green's function is
G(r, t) = c H(ct - r) / (2 pi sqrt(c^2 t^2 - r^2)).  A source value q^n on
one grid node stands for f = h^2 q(t) delta(x) (a grid function of point
values integrates to its sum times the cell area), so with
tau = (r/c) cosh(s) the trace at distance r is
u(r, t) = h^2/(2 pi) * integral_0^{acosh(ct/r)} q(t - (r/c) cosh s) ds.
Injection scale, injection time level and receiver time level all enter the
comparison: a lost factor or a shift by one step fails it.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle

C, F0, R = 1500.0, 10.0, 200.0


def _ricker(t):
    a = (np.pi * F0 * (t - 1.0 / F0)) ** 2
    return (1 - 2 * a) * np.exp(-a)


def _green_trace(h, dt, nt, r):
    t = np.arange(nt) * dt
    out = np.zeros(nt)
    for i, tt in enumerate(t):
        if C * tt > r:
            smax = np.arccosh(C * tt / r)
            out[i] = h * h / (2 * np.pi) * quad(lambda s: _ricker(tt - r / C * np.cosh(s)), 0.0,
                                                smax, limit=200)[0]
    return out


def _relerr(h, order, shift=0):
    """Relative L2 error of three receivers at distance R (axis, axis,
    diagonal) over 0.6 s, on a grid large enough that no reflection returns."""
    dt = 0.4 * h / C
    nt = int(0.6 / dt)
    n = int(round(3000.0 / h)) + 1
    ctr = (n - 1) // 2 * h
    q = _ricker(np.arange(nt) * dt).astype(np.float32).reshape(nt, 1)
    if shift:
        q = np.roll(q, shift, axis=0)
    rec = np.array([[ctr + R, ctr], [ctr, ctr + R], [ctr + 0.6 * R, ctr + 0.8 * R]])
    m = np.full((n, n), 1.0 / C ** 2, dtype=np.float32)
    d = oracle.forward((n, n), (h, h), order, dt, nt, m, None, np.array([[ctr, ctr]]), q, rec)["d"]
    ref = _green_trace(h, dt, nt, R)
    return max(np.linalg.norm(d[:, k] - ref) / np.linalg.norm(ref) for k in range(3))


def test_point_source_matches_2d_greens_function():
    e10 = _relerr(10.0, 4)
    e5 = _relerr(5.0, 4)
    # about 15 points per peak wavelength at h = 10 m: dispersion at the percent level
    assert e10 < 2.5e-2, e10
    # the discrepancy is discretisation error: it falls under refinement
    assert e5 < e10 / 2, (e5, e10)
    # higher order in space at the same h stays at the same level (time error dominates)
    assert _relerr(10.0, 8) < 2.5e-2


def test_one_step_time_shift_is_detected():
    # the pin's own resolution: a source one step late (a wrong time level) fails it
    assert _relerr(10.0, 4, shift=1) > 5e-2
