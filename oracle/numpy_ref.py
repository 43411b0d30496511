"""Second, independent statement of the forward scheme in NumPy (tiny grids).

TEST INFRASTRUCTURE ONLY.  Written separately from ``wave_oracle.c`` (array
slicing over a zero-padded field instead of bounds-checked loops, weights from
an exact Vandermonde solve instead of the closed form) so that the two can
check each other.  FP64 throughout.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def fd_weights_vandermonde(order: int):
    """Exact weights of the (order+1)-point central 2nd derivative, solving
    sum_j c_j j^p = 2 [p == 2] for p = 0..order with rational arithmetic.
    Returns Fractions c_0..c_k (c_{-j} = c_j)."""
    k = order // 2
    offs = list(range(-k, k + 1))
    n = len(offs)
    A = [[Fraction(o) ** p for o in offs] for p in range(n)]
    b = [Fraction(2 if p == 2 else 0) for p in range(n)]
    # Gauss-Jordan elimination over the rationals
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    sol = [M[i][n] for i in range(n)]
    return [sol[k + j] for j in range(k + 1)]


def laplacian(u, spacing, order):
    """Sum over axes of the order-``order`` central 2nd difference, zero outside."""
    c = [float(x) for x in fd_weights_vandermonde(order)]
    k = order // 2
    nd = u.ndim
    up = np.pad(u, k)
    core = tuple(slice(k, k + s) for s in u.shape)
    out = np.zeros_like(u, dtype=np.float64)
    for a in range(nd):
        acc = np.zeros_like(out)
        for j in range(-k, k + 1):
            sl = list(core)
            sl[a] = slice(k + j, k + j + u.shape[a])
            acc += c[abs(j)] * up[tuple(sl)]
        out += acc / (spacing[a] ** 2)
    return out


def interp_weights(shape, spacing, pts):
    """Per point: list of (multi-index, weight) over the 2^d cell corners."""
    res = []
    for p in np.asarray(pts, dtype=np.float64):
        base, frac = [], []
        for a, n in enumerate(shape):
            if p[a] < 0 or p[a] > (n - 1) * spacing[a]:
                raise ValueError("point outside the grid")
            x = min(p[a] / spacing[a], n - 1)
            i = min(int(np.floor(x)), n - 2)
            base.append(i)
            frac.append(x - i)
        corners = []
        for bits in np.ndindex(*([2] * len(shape))):
            w = 1.0
            for a, bt in enumerate(bits):
                w *= frac[a] if bt else 1.0 - frac[a]
            corners.append((tuple(b + bt for b, bt in zip(base, bits)), w))
        res.append(corners)
    return res


def forward(shape, spacing, order, dt, nt, m, eta, src, q, rec):
    """Forward run from rest; returns (d [nt][nrec], u^nt)."""
    m = np.asarray(m, dtype=np.float64).reshape(shape)
    eta = np.zeros(shape) if eta is None else np.asarray(eta, dtype=np.float64).reshape(shape)
    a = m + 0.5 * dt * eta
    b = m - 0.5 * dt * eta
    S = interp_weights(shape, spacing, src)
    R = interp_weights(shape, spacing, rec)
    q = np.asarray(q, dtype=np.float64).reshape(nt, len(S))
    u_old = np.zeros(shape)
    u = np.zeros(shape)
    d = np.zeros((nt, len(R)))
    for n in range(nt):
        for r, corners in enumerate(R):
            d[n, r] = sum(w * u[idx] for idx, w in corners)
        u_new = (2.0 * m * u - b * u_old + dt * dt * laplacian(u, spacing, order)) / a
        for s, corners in enumerate(S):
            for idx, w in corners:
                u_new[idx] += dt * dt * q[n, s] * w / a[idx]
        u_old, u = u, u_new
    return d, u
