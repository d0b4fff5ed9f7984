"""numpy wrappers of the oracle's C primitives on one uniform periodic level.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fields are float64 arrays shaped (3, nz, ny, nx) (x fastest); resistivity is
(nz, ny, nx).  All cells are cubes of width ``h``; boundaries are periodic
(every test of the paper is periodic).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import build_oracle

_lib = None
_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_oracle.build())
        for name, args in {
            "oref_flux": [_I, _I, _I, _D, _P, _P, _P],
            "oref_div": [_I, _I, _I, _D, _P, _P],
            "oref_apply": [_I, _I, _I, _D, _P, _P, _D, _P],
            "oref_residual": [_I, _I, _I, _D, _P, _P, _P, _D, _P],
            "oref_alpha": [_I, _I, _I, _D, _P, _D, _P],
            "oref_rb_halfsweep": [_I, _I, _I, _D, _P, _P, _P, _D, _I],
            "oref_restrict": [_I, _I, _I, _I, _P, _P],
            "oref_prolong_add": [_I, _I, _I, _I, _P, _P],
        }.items():
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = None
        _lib.oref_threads.argtypes = []
        _lib.oref_threads.restype = ctypes.c_int
        _lib.oref_set_threads.argtypes = [_I]
        _lib.oref_set_threads.restype = None
    return _lib


def threads() -> int:
    """OpenMP threads of the C primitives."""
    return int(lib().oref_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the C primitives (timing only)."""
    lib().oref_set_threads(int(n))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(a: np.ndarray):
    nz, ny, nx = a.shape[-3:]
    return nx, ny, nz


def flux(B, eta, h):
    """Face fluxes F[d, c] (eqs. 4-6 with 9-11): component c of F_d on the face
    between cell p and p + e_d.  Shape (3, 3, nz, ny, nx)."""
    B, eta = _c(B), _c(eta)
    F = np.empty((3, 3) + B.shape[1:])
    lib().oref_flux(*_dims(B), h, _p(B), _p(eta), _p(F))
    return F


def div(F, h):
    """Flux divergence (eq. 8).  Shape (3, nz, ny, nx)."""
    F = _c(F)
    out = np.empty((3,) + F.shape[2:])
    lib().oref_div(*_dims(F), h, _p(F), _p(out))
    return out


def apply(B, eta, h, coef):
    """B + coef * div F(B): the operator L (eq. 13) for coef = lambda dt."""
    B, eta = _c(B), _c(eta)
    out = np.empty_like(B)
    lib().oref_apply(*_dims(B), h, _p(B), _p(eta), coef, _p(out))
    return out


def source(b, eta, h, dt, lam=0.5):
    """S = b - (1 - lambda) dt div f(b) (eq. 14)."""
    return apply(b, eta, h, -(1.0 - lam) * dt)


def residual(B, S, eta, h, lam_dt):
    """R = S - L B (eq. 20)."""
    B, S, eta = _c(B), _c(S), _c(eta)
    R = np.empty_like(B)
    lib().oref_residual(*_dims(B), h, _p(B), _p(S), _p(eta), lam_dt, _p(R))
    return R


def alpha(eta, h, lam_dt):
    """alpha_c of eqs. (21)-(23).  Shape (3, nz, ny, nx)."""
    eta = _c(eta)
    out = np.empty((3,) + eta.shape)
    lib().oref_alpha(*_dims(eta), h, _p(eta), lam_dt, _p(out))
    return out


def rb_halfsweep(B, S, eta, h, lam_dt, colour):
    """One red (colour 0) or black (colour 1) half-sweep of eq. (19); returns a
    new array.  Colour of cell (i, j, k) is (i + j + k) mod 2 in level indices."""
    B = _c(B).copy()
    S, eta = _c(S), _c(eta)
    lib().oref_rb_halfsweep(*_dims(B), h, _p(B), _p(S), _p(eta), lam_dt, int(colour))
    return B


def colour_classes(shape, ordering=0):
    """Colour class of every cell (i, j, k) of a (nz, ny, nx) level, in level
    indices.  ordering 0: the paper's red (0) and black (1), (i + j + k) mod 2.
    ordering 1: four classes ((i + j) mod 2) + 2 ((j + k) mod 2), an ordering
    the paper does not use, under which no two cells of a class share a
    stencil term."""
    k, j, i = np.indices(shape)
    if ordering == 0:
        return (i + j + k) % 2
    return (i + j) % 2 + 2 * ((j + k) % 2)


def class_update(B, S, eta, h, lam_dt, classes, m):
    """The update of eq. (19), B_c += R_c / (1 + alpha_c) with R = S - L B of
    the incoming field, on the cells of class m only; returns a new array."""
    B = _c(B)
    R = residual(B, S, eta, h, lam_dt)
    al = alpha(eta, h, lam_dt)
    return np.where((classes == m)[None], B + R / (1.0 + al), B)


def smooth(B, S, eta, h, lam_dt, nsweeps, ordering=0):
    """``nsweeps`` sweeps: red-black (red half first), or with ordering 1 the
    four classes of ``colour_classes`` in the order 0, 1, 2, 3."""
    if ordering == 0:
        for _ in range(nsweeps):
            B = rb_halfsweep(B, S, eta, h, lam_dt, 0)
            B = rb_halfsweep(B, S, eta, h, lam_dt, 1)
        return B
    classes = colour_classes(np.shape(eta), ordering)
    for _ in range(nsweeps):
        for m in range(4):
            B = class_update(B, S, eta, h, lam_dt, classes, m)
    return B


def restrict(fine):
    """Averaging restriction: mean of the 8 children.  Works on (ncomp, z, y, x)
    or (z, y, x) arrays."""
    fine = _c(fine)
    scalar = fine.ndim == 3
    f = fine[None] if scalar else fine
    nc = f.shape[0]
    nzf, nyf, nxf = f.shape[1:]
    assert nxf % 2 == 0 and nyf % 2 == 0 and nzf % 2 == 0
    out = np.empty((nc, nzf // 2, nyf // 2, nxf // 2))
    lib().oref_restrict(nxf // 2, nyf // 2, nzf // 2, nc, _p(f), _p(out))
    return out[0] if scalar else out


def prolong(coarse, fine=None):
    """Cell-centred trilinear prolongation (27/9/3/1 over 64), added to
    ``fine`` (zeros if None).  Returns the new fine array."""
    coarse = _c(coarse)
    scalar = coarse.ndim == 3
    c = coarse[None] if scalar else coarse
    nc, nzc, nyc, nxc = c.shape
    if fine is None:
        out = np.zeros((nc, 2 * nzc, 2 * nyc, 2 * nxc))
    else:
        out = _c(fine).copy()
        out = out[None] if scalar else out
    lib().oref_prolong_add(nxc, nyc, nzc, nc, _p(c), _p(out))
    return out[0] if scalar else out
