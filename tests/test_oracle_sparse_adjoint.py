"""Pins of the oracle's sparse-point operators, adjoint and gradient.

* multilinear interpolation reproduces multilinear functions exactly, its
  weights are a partition of unity, the upper edge clamps, outside is ERANGE;
* a source on a grid node is the same as a dense forcing at that node;
* the first two recorded samples have a closed form (d^0 = 0, d^1 from the
  first injection);
* the adjoint is the transpose of the forward map q -> d: dot test (the
  paper's validation, equation "eqn:adjtest") and, on a tiny case, the full
  matrices;
* the gradient passes a Taylor test and equals its summation-by-parts form.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1609_03361_amd import synth


@pytest.mark.parametrize("shape", [(7, 9), (5, 6, 8)])
def test_multilinear_exactness_and_partition_of_unity(shape):
    rng = np.random.default_rng(1)
    ndim = len(shape)
    spacing = tuple(rng.uniform(5, 15, ndim))
    ext = np.array([(n - 1) * h for n, h in zip(shape, spacing)])
    pts = rng.uniform(0, 1, (50, ndim)) * ext
    pts[0] = ext
    pts[1] = 0
    corner, w = oracle.sparse_weights(shape, spacing, pts)
    assert np.all(w >= -1e-15)
    assert np.max(np.abs(w.sum(axis=1) - 1.0)) < 1e-14
    coef = rng.standard_normal(1 << ndim)
    grids = np.meshgrid(*[np.arange(n) * h for n, h in zip(shape, spacing)], indexing="ij")

    def f(coords):          # sum over subsets S of axes of coef_S prod_{a in S} x_a
        out = 0.0
        for s in range(1 << ndim):
            term = coef[s]
            for a in range(ndim):
                if (s >> a) & 1:
                    term = term * coords[a]
            out = out + term
        return out

    field = f(grids).ravel()
    sampled = np.sum(w * field[corner], axis=1)
    exact = f([pts[:, a] for a in range(ndim)])
    assert np.max(np.abs(sampled - exact)) < 1e-12 * np.max(np.abs(exact))


def test_upper_edge_clamp_and_range():
    shape, spacing = (6, 5), (10.0, 10.0)
    corner, w = oracle.sparse_weights(shape, spacing, [[50.0, 40.0]])
    # only the (i0+1, k0+1) = (5, 4) corner carries weight, with i0 = n-2
    assert corner[0, 3] == 5 * 5 + 4 and w[0, 3] == 1.0
    assert np.all(w[0, :3] == 0.0)
    for bad in ([[-1e-9, 0.0]], [[50.0 + 1e-6, 0.0]], [[0.0, 40.0 + 1e-6]]):
        with pytest.raises(oracle.OracleError) as e:
            oracle.sparse_weights(shape, spacing, bad)
        assert e.value.code == -3


def test_grid_node_source_equals_dense_forcing():
    p = synth.random_problem((10, 12), 4, 20, seed=2, nsrc=1, nrec=3)
    node = (4, 7)
    src = np.array([[node[0] * p.spacing[0], node[1] * p.spacing[1]]])
    a = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, src, p.q, p.rec)
    pat = np.zeros(p.shape)
    pat[node] = 1.0
    b = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, None, None, p.rec,
                       force_pat=pat[None], force_t=p.q.astype(np.float64))
    assert np.max(np.abs(a["u"] - b["u"])) <= 1e-13 * np.max(np.abs(b["u"]))
    assert np.max(np.abs(a["d"] - b["d"])) <= 1e-13 * np.max(np.abs(b["d"]))


@pytest.mark.parametrize("shape", [(9, 8), (6, 7, 5)])
def test_first_samples_closed_form(shape):
    """From rest: d^0 = 0 and u^1 = dt^2 sum_s q^0_s w_{s,c} / a at the source
    corners, so d^1_r = sum_c w_{r,c} u^1[corner]."""
    p = synth.random_problem(shape, 8, 2, seed=4, nsrc=3, nrec=6)
    r = oracle.forward(p.shape, p.spacing, p.order, p.dt, 2, p.m, p.eta, p.src, p.q, p.rec)
    assert np.all(r["d"][0] == 0.0)
    a = p.m.astype(np.float64).ravel() + 0.5 * p.dt * p.eta.astype(np.float64).ravel()
    sc, sw = oracle.sparse_weights(p.shape, p.spacing, p.src)
    u1 = np.zeros(a.size)
    for s in range(sc.shape[0]):
        for c in range(sc.shape[1]):
            u1[sc[s, c]] += p.dt ** 2 * float(p.q[0, s]) * sw[s, c] / a[sc[s, c]]
    rc, rw = oracle.sparse_weights(p.shape, p.spacing, p.rec)
    d1 = np.sum(rw * u1[rc], axis=1)
    assert np.max(np.abs(r["d"][1] - d1)) <= 1e-14 * np.max(np.abs(d1))


@pytest.mark.parametrize("shape,order", [((30, 26), 2), ((28, 31), 8), ((26, 24), 16),
                                         ((14, 12, 13), 4), ((12, 13, 11), 12)])
def test_dot_product(shape, order):
    """<F q, d> = <q, F^T d> for random q and d (the paper's adjoint test)."""
    p = synth.random_problem(shape, order, 60, seed=order, nsrc=3, nrec=9)
    rng = np.random.default_rng(99)
    dy = rng.standard_normal((p.nt, p.rec.shape[0]))
    Fq = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q,
                        p.rec, want_final=False)["d"]
    FTd = oracle.adjoint(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.rec, dy,
                         p.src)["qadj"]
    lhs = np.sum(Fq * dy)
    rhs = np.sum(p.q.astype(np.float64) * FTd)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_adjoint_matrix_is_forward_transpose():
    p = synth.random_problem((8, 9), 4, 6, seed=8, nsrc=2, nrec=3)
    nt, ns, nr = p.nt, 2, 3
    F = np.zeros((nt * nr, nt * ns))
    for k in range(nt * ns):
        q = np.zeros(nt * ns)
        q[k] = 1.0
        F[:, k] = oracle.forward(p.shape, p.spacing, p.order, p.dt, nt, p.m, p.eta, p.src, q,
                                 p.rec, want_final=False)["d"].ravel()
    FT = np.zeros((nt * ns, nt * nr))
    for k in range(nt * nr):
        d = np.zeros(nt * nr)
        d[k] = 1.0
        FT[:, k] = oracle.adjoint(p.shape, p.spacing, p.order, p.dt, nt, p.m, p.eta, p.rec, d,
                                  p.src)["qadj"].ravel()
    assert np.max(np.abs(F)) > 0
    assert np.max(np.abs(F.T - FT)) <= 1e-14 * np.max(np.abs(F))


def _grad_problem(shape=(22, 20), order=8, nt=80):
    p = synth.random_problem(shape, order, nt, seed=21, nsrc=2, nrec=11)
    rng = np.random.default_rng(5)
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(shape), 2.0)
    dm *= 0.05 * float(np.mean(p.m)) / np.max(np.abs(dm))
    m_true = p.m.astype(np.float64) + dm
    d_obs = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, m_true, p.eta, p.src, p.q,
                           p.rec, want_final=False)["d"]
    return p, d_obs


def test_gradient_plain_equals_summation_by_parts():
    p, d_obs = _grad_problem()
    r = oracle.gradient(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                        d_obs, sbp=True)
    assert np.max(np.abs(r["grad"] - r["grad_sbp"])) <= 1e-12 * np.max(np.abs(r["grad"]))


@pytest.mark.parametrize("shape", [(22, 20), (10, 9, 11)])
def test_gradient_taylor(shape):
    """|J(m + h dm) - J(m) - h <g, dm>| falls by 4x per halving of h."""
    p, d_obs = _grad_problem(shape, nt=70)
    r = oracle.gradient(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                        d_obs)
    g, J0 = r["grad"], r["J"]
    rng = np.random.default_rng(6)
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(shape), 1.5)
    dm *= 0.02 * float(np.mean(p.m)) / np.max(np.abs(dm))
    m = p.m.astype(np.float64)
    rem1, rem0 = [], []
    for k in range(5):
        h = 2.0 ** -k
        d = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, m + h * dm, p.eta, p.src,
                           p.q, p.rec, want_final=False)["d"]
        J = 0.5 * np.sum((d - d_obs) ** 2)
        rem0.append(abs(J - J0))
        rem1.append(abs(J - J0 - h * np.sum(g * dm)))
    s1 = [math.log2(rem1[i] / rem1[i + 1]) for i in range(4)]
    s0 = [math.log2(rem0[i] / rem0[i + 1]) for i in range(4)]
    assert all(abs(s - 2.0) < 0.1 for s in s1), (s1, rem1)
    assert all(abs(s - 1.0) < 0.1 for s in s0), (s0, rem0)
