"""Full-waveform-inversion iterations around the gradient path.

The paper's motivating workflow (Section "Seismic Inversion Example": the
forward and adjoint operators serve adjoint-based inversion) in its plainest
form: steepest descent on the squared slowness m with a backtracking
(Armijo) line search on the misfit, summed over shots.  Every wave
propagation, misfit and gradient runs in libwave.so (wave_forward,
wave_gradient); this module only sums per-shot results, scales the search
direction and keeps m inside velocity bounds.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import api

__all__ = ["FWIState", "misfit", "misfit_and_gradient", "fwi_iteration"]


@dataclass
class FWIState:
    """Shots (Geometry, wavelets q, observed data), fixed damping, bounds."""
    shots: list                  # [(Geometry, q, d_obs)]
    eta: torch.Tensor | None
    vmin: float
    vmax: float
    ckpt_every: int = 20
    ckpt_dtype: str = "fp32"
    mask: torch.Tensor | None = None   # multiplies the gradient (e.g. 0 in the sponge)
    history: list = field(default_factory=list)

    @property
    def m_bounds(self):
        return 1.0 / (self.vmax * self.vmax), 1.0 / (self.vmin * self.vmin)


def misfit(state: FWIState, m: torch.Tensor) -> float:
    """J(m) = 1/2 sum over shots of |d(m) - d_obs|^2 (forward runs and the
    library's misfit reduction only)."""
    J = 0.0
    for geom, q, d_obs in state.shots:
        d = api.forward(geom, m, state.eta, q)
        J += float(api.misfit(d, d_obs))
    return J


def misfit_and_gradient(state: FWIState, m: torch.Tensor):
    """J(m) and dJ/dm summed over shots (checkpointed adjoint-state gradient)."""
    g = torch.zeros_like(m)
    J = 0.0
    for geom, q, d_obs in state.shots:
        Js, gs = api.gradient(geom, m, state.eta, q, d_obs, ckpt_every=state.ckpt_every,
                              ckpt_dtype=state.ckpt_dtype)
        g += gs
        J += float(Js)
    if state.mask is not None:
        g *= state.mask
    return J, g


def fwi_iteration(state: FWIState, m: torch.Tensor, step: float = 0.05, shrink: float = 0.5,
                  c1: float = 1e-4, max_tries: int = 6):
    """One steepest-descent iteration.  The direction -g is scaled so that its
    largest entry is `step` times the largest |m|; the step is halved until
    the Armijo condition J(m + a p) <= J(m) + c1 a <g, p> holds.  Returns
    (m_new, J_new, accepted step a)."""
    J0, g = misfit_and_gradient(state, m)
    p = -g * (step * float(m.abs().max()) / max(float(g.abs().max()), 1e-30))
    gp = float((g.double() * p.double()).sum())
    lo, hi = state.m_bounds
    a = 1.0
    for _ in range(max_tries):
        m_try = (m + a * p).clamp(lo, hi).contiguous()
        J = misfit(state, m_try)
        if J <= J0 + c1 * a * gp:
            state.history.append({"J0": J0, "J": J, "a": a})
            return m_try, J, a
        a *= shrink
    state.history.append({"J0": J0, "J": J0, "a": 0.0})
    return m, J0, 0.0
