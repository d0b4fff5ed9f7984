"""Explicit comparison scheme of section 3.3 (FP64, plain numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper compares its implicit scheme with an explicit one that advances in
time by a predictor-corrector method with a central-difference stencil, second
order in time and space.  Reading: Heun's predictor-corrector (the explicit
trapezoidal rule) on the same flux divergence as the implicit operator
(eqs. 8-11):

    B* = B - dt div F(B)                       (predictor, forward Euler)
    B' = B - dt/2 (div F(B) + div F(B*))       (corrector, trapezoidal)

On an AMR hierarchy every stage uses the composite flux divergence (covered
cells restricted from their children, coarse-fine ghosts interpolated, fluxes
refluxed) and the covered cells of the result are the mean of their children.
"""
from __future__ import annotations

from . import ref


def heun_steps(b, eta, h, dt, nsteps):
    """``nsteps`` steps on one periodic uniform level; b: (3, nz, ny, nx)."""
    B = b.copy()
    for _ in range(nsteps):
        D = ref.div(ref.flux(B, eta, h), h)
        Bp = B - dt * D
        Dp = ref.div(ref.flux(Bp, eta, h), h)
        B = B - 0.5 * dt * (D + Dp)
    return B


def heun_steps_amr(comp, Bs, etas, dt, nsteps):
    """``nsteps`` steps on the composite leaf cells of an AMR hierarchy
    (``comp``: an amr.Composite); Bs, etas: dense per-level arrays."""
    Bs = comp.average_down(Bs)
    for _ in range(nsteps):
        D = comp.divF(Bs, etas)
        Bp = comp.average_down([Bs[l] - dt * D[l] for l in range(comp.L)])
        Dp = comp.divF(Bp, etas)
        Bs = comp.average_down([Bs[l] - 0.5 * dt * (D[l] + Dp[l]) for l in range(comp.L)])
    return Bs
