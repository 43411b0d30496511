"""Pins of the oracle's diffusion (Section "2D Diffusion Example").

* With order 2, equal spacing and the time step of equation
  "eqn:diffusion_dt", one step is exactly the generated kernel the paper
  prints: 0.25 times the sum of the four neighbours, no centre term
  (tests/golden/paper_diffusion_kernel.txt);
* Dirichlet sine modes of the order-2 operator decay by exactly
  (1 - dt a lambda) per step.
"""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_one_step_is_the_paper_generated_kernel():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_diffusion_kernel.txt"))
            if l.strip() and not l.startswith("#")]
    taps = {(int(a), int(b)): float(w) for a, b, w in rows}
    rng = np.random.default_rng(0)
    n, h, alpha = 24, 0.001, 0.5
    dt = h ** 2 * h ** 2 / (2 * alpha * (h ** 2 + h ** 2))       # eqn:diffusion_dt
    u0 = rng.standard_normal((n, n))
    got = oracle.diffusion((n, n), (h, h), 2, dt, 1, np.full((n, n), alpha), u0)
    up = np.pad(u0, 1)
    want = sum(w * up[1 + a:1 + a + n, 1 + b:1 + b + n] for (a, b), w in taps.items())
    assert (0, 0) not in taps
    assert np.max(np.abs(got - want)) < 1e-13


def test_sine_mode_decay():
    shape, spacing = (15, 11), (0.1, 0.2)
    j = (3, 2)
    a, nt = 0.7, 25
    lam = sum(4.0 / hh ** 2 * math.sin(math.pi * jj / (2 * (nn + 1))) ** 2
              for nn, hh, jj in zip(shape, spacing, j))
    lam_max = sum(4.0 / hh ** 2 for hh in spacing)     # stable for every mode: dt a lam_max < 2
    dt = 1.5 / (a * lam_max)
    phi = np.outer(np.sin(math.pi * j[0] * np.arange(1, shape[0] + 1) / (shape[0] + 1)),
                   np.sin(math.pi * j[1] * np.arange(1, shape[1] + 1) / (shape[1] + 1)))
    got = oracle.diffusion(shape, spacing, 2, dt, nt, np.full(shape, a), phi)
    assert np.max(np.abs(got - (1 - dt * a * lam) ** nt * phi)) < 1e-13
