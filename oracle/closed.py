"""Closed forms that pin the oracle (constant resistivity, periodic box).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For B = v exp(i k.x) on a periodic grid of cubic cells of width h and constant
eta, the discrete flux divergence of eqs. (8)-(11) is eta M(k) v with

    M = diag_c( sum_{d != c} s_d^2 + cc_c^2 ) - cc cc^T,
    s_d  = (2/h) sin(k_d h / 2)      (compact difference across a face, eq. 9)
    cc_d = sin(k_d h) / h            (four-point transverse difference, eq. 10)

(derived by inserting the Fourier mode into eqs. 8-10).  One step of eq. (7)
multiplies each Fourier coefficient by
    G(k) = (I + lam dt eta M)^{-1} (I - (1 - lam) dt eta M).
"""
from __future__ import annotations

import numpy as np


def symbol(kx, ky, kz, h):
    """M(k) for arrays of wavenumbers: shape (..., 3, 3)."""
    k = np.stack(np.broadcast_arrays(kx, ky, kz), axis=-1).astype(float)
    s = (2.0 / h) * np.sin(k * h / 2.0)
    cc = np.sin(k * h) / h
    s2 = s * s
    diag = s2.sum(-1)[..., None] - s2 + cc * cc
    M = -cc[..., :, None] * cc[..., None, :]
    idx = np.arange(3)
    M[..., idx, idx] += diag
    return M


def cn_exact(b, eta0, h, dt, lam=0.5, nsteps=1):
    """Exact solution of ``nsteps`` steps of the discrete scheme (eq. 7) for
    constant resistivity eta0, by FFT.  b: (3, nz, ny, nx)."""
    _, nz, ny, nx = b.shape
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    M = eta0 * symbol(KX, KY, KZ, h)
    I = np.eye(3)
    G = np.linalg.solve(I + lam * dt * M, I - (1 - lam) * dt * M)
    Gn = np.linalg.matrix_power(G, nsteps)
    bh = np.fft.fftn(b, axes=(1, 2, 3))
    bh = np.moveaxis(bh, 0, -1)[..., None]
    out = (Gn @ bh)[..., 0]
    return np.real(np.fft.ifftn(np.moveaxis(out, -1, 0), axes=(1, 2, 3)))


def heat_factor(kx, ky, h, eta0, dt, lam=0.5):
    """Per-step amplification of B_z = sin(k.r) with k in the x-y plane: the
    scheme reduces to the 5-point heat equation, g = (1-(1-lam) dt mu) /
    (1 + lam dt mu) with mu = eta (s_x^2 + s_y^2)."""
    mu = eta0 * ((2 / h * np.sin(kx * h / 2)) ** 2 + (2 / h * np.sin(ky * h / 2)) ** 2)
    return (1 - (1 - lam) * dt * mu) / (1 + lam * dt * mu)


def continuum_decay(k2, eta0, t):
    """exp(-eta |k|^2 t), the exact continuum decay of a Fourier mode (eq. 25)."""
    return np.exp(-eta0 * k2 * t)


def heun_exact(b, eta0, h, dt, nsteps=1):
    """``nsteps`` steps of the explicit predictor-corrector scheme for constant
    resistivity, by FFT: each Fourier coefficient is multiplied by
    E(k) = I - dt M + (dt M)^2 / 2 per step (B* = B - dt M B, then
    B' = B - dt/2 (M B + M B*))."""
    _, nz, ny, nx = b.shape
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    A = dt * eta0 * symbol(KX, KY, KZ, h)
    I = np.eye(3)
    E = I - A + 0.5 * (A @ A)
    En = np.linalg.matrix_power(E, nsteps)
    bh = np.fft.fftn(b, axes=(1, 2, 3))
    bh = np.moveaxis(bh, 0, -1)[..., None]
    out = (En @ bh)[..., 0]
    return np.real(np.fft.ifftn(np.moveaxis(out, -1, 0), axes=(1, 2, 3)))


def semidiscrete_exact(b, eta0, h, t):
    """The space-discrete, time-exact solution exp(-t eta M) b for constant
    resistivity (M is symmetric per wavevector: eigendecomposition)."""
    _, nz, ny, nx = b.shape
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    w, V = np.linalg.eigh(eta0 * symbol(KX, KY, KZ, h))
    G = V @ (np.exp(-t * w)[..., None] * np.swapaxes(V, -1, -2))
    bh = np.fft.fftn(b, axes=(1, 2, 3))
    bh = np.moveaxis(bh, 0, -1)[..., None]
    out = (G @ bh)[..., 0]
    return np.real(np.fft.ifftn(np.moveaxis(out, -1, 0), axes=(1, 2, 3)))
