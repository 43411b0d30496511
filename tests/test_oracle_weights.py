"""Pins of the oracle's finite-difference weights and Laplacian.

The weights are checked against (a) the expansion the paper prints for
space_order=2 (Section "High-level API"), (b) an exact rational Vandermonde
solve written independently in ``oracle.numpy_ref``, and (c) polynomial
exactness: the order-2k stencil differentiates x^p exactly for p <= 2k+1 and
not for p = 2k+2.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import numpy_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORDERS = list(range(2, 18, 2))


def test_order2_matches_paper_expansion():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_dx2_order2.txt"))
            if l.strip() and not l.startswith("#")]
    printed = {int(o): float(w) for o, w in rows}
    c = oracle.fd_weights(2)
    assert c[0] == printed[0]
    assert c[1] == printed[1] == printed[-1]


@pytest.mark.parametrize("order", ORDERS)
def test_closed_form_equals_exact_vandermonde(order):
    exact = numpy_ref.fd_weights_vandermonde(order)
    c = oracle.fd_weights(order)
    for j, e in enumerate(exact):
        assert abs(c[j] - float(e)) <= 4e-16 * max(1.0, abs(float(e))), (order, j)


@pytest.mark.parametrize("order", ORDERS)
def test_vandermonde_moments_are_those_of_a_second_derivative(order):
    """sum_j c_j j^p = 2 [p == 2] for p <= 2k+1 (p odd vanish by symmetry)
    and the first non-zero error moment is at p = 2k+2."""
    k = order // 2
    c = numpy_ref.fd_weights_vandermonde(order)
    full = {j: c[abs(j)] for j in range(-k, k + 1)}
    for p in range(0, 2 * k + 2):
        mom = sum(w * Fraction(j) ** p for j, w in full.items())
        assert mom == (2 if p == 2 else 0), (order, p)
    p = 2 * k + 2
    mom = sum(w * Fraction(j) ** p for j, w in full.items())
    assert mom != 0


@pytest.mark.parametrize("order", [2, 4, 8, 12, 16])
def test_laplacian_exact_on_polynomials(order):
    """oracle.laplacian on u = x^p (constant along z): exact for p <= order+1;
    at p = order+2 the error is the constant sum_j c_j j^p (the first
    non-vanishing moment, computed exactly).  Checked away from the zero halo:
    x in [k, n-k) and the middle z column of a (2k+1)-wide z axis."""
    k = order // 2
    n = 4 * k + 3
    shape = (n, 2 * k + 1)
    x = np.arange(n, dtype=np.float64) - (n - 1) / 2
    scale = float(np.max(np.abs(x)))
    interior = slice(k, n - k)
    for p in range(0, order + 3):
        u = np.repeat(((x / scale) ** p)[:, None], 2 * k + 1, axis=1)
        lu = oracle.laplacian(shape, (1.0, 1.0), order, u)
        exact = (p * (p - 1) * x ** (p - 2) / scale ** p) if p >= 2 else 0 * x
        err = np.max(np.abs(lu[interior, k] - exact[interior]))
        if p <= order + 1:
            assert err < 1e-11, (order, p, err)
        else:
            c = numpy_ref.fd_weights_vandermonde(order)
            mom = float(sum(c[abs(j)] * Fraction(j) ** p for j in range(-k, k + 1)))
            dev = lu[interior, k] - exact[interior]
            assert np.allclose(dev, mom / scale ** p, rtol=1e-2, atol=0), (order, p)


@pytest.mark.parametrize("ndim,order", [(2, 2), (2, 8), (3, 4), (3, 16)])
def test_laplacian_symmetric_negative_definite(ndim, order):
    """The assembled operator (zero extension outside the grid) is symmetric
    and negative definite; its spectrum is bounded by sum_a S/h_a^2 with
    S = sum |c_j| over the full stencil (the Nyquist symbol)."""
    rng = np.random.default_rng(order)
    shape = (5, 4) if ndim == 2 else (4, 3, 5)
    spacing = tuple(rng.uniform(0.5, 2.0, ndim))
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        A[:, i] = oracle.laplacian(shape, spacing, order, e.reshape(shape)).ravel()
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(A)
    assert ev.max() < 0
    c = oracle.fd_weights(order)
    S = abs(c[0]) + 2 * np.sum(np.abs(c[1:]))
    assert -ev.min() <= sum(S / h ** 2 for h in spacing) * (1 + 1e-12)


@pytest.mark.parametrize("ndim,order", [(2, 4), (3, 8), (3, 16)])
def test_laplacian_matches_numpy_restatement(ndim, order):
    rng = np.random.default_rng(7)
    shape = (9, 11) if ndim == 2 else (9, 7, 10)
    spacing = tuple(rng.uniform(5.0, 15.0, ndim))
    u = rng.standard_normal(shape)
    a = oracle.laplacian(shape, spacing, order, u)
    b = numpy_ref.laplacian(u, spacing, order)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
