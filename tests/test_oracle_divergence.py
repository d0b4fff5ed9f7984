"""The central-difference divergence of B under the scheme (eqs. 7-11).

The flux form does not keep div_c B = sum_c (B_c(p + e_c) - B_c(p - e_c)) / 2h
at zero for general fields, so nothing here asserts invariance on generic
data.  What is fixed: (i) a field B = (0, 0, B_z(x, y)) with eta(x, y) stays
of that form under the operator, exactly, so its divergence stays zero; (ii)
for a single discretely divergence-free Fourier mode the divergence one step
creates has a closed form from the symbol M(k), and it is second order in h.
"""
import numpy as np
import pytest

from oracle import closed, mg, ref


def div_c(B, h):
    out = np.zeros(B.shape[1:])
    for c, ax in enumerate((2, 1, 0)):
        out += (np.roll(B[c], -1, ax) - np.roll(B[c], 1, ax)) / (2 * h)
    return out


def test_two_coordinate_field_stays_in_its_subspace():
    """L maps (0, 0, B_z(x, y)) to (0, 0, g(x, y)) bit for bit when eta depends
    on x and y only: the x and y fluxes of the x and y components vanish and
    every z-plane computes the same numbers.  The solved step keeps the form
    to rounding."""
    nz, ny, nx, h = 4, 8, 6, 0.11
    rng = np.random.default_rng(3)
    eta = np.broadcast_to(np.exp(rng.uniform(-1, 1, (1, ny, nx))), (nz, ny, nx)).copy()
    B = np.zeros((3, nz, ny, nx))
    B[2] = rng.standard_normal((1, ny, nx))
    out = ref.apply(B, eta, h, 0.37)
    assert not out[0].any() and not out[1].any()
    assert all(np.array_equal(out[2][k], out[2][0]) for k in range(nz))
    assert not div_c(out, h).any()
    dt = 10 * h * h / eta.max()
    S = ref.source(B, eta, h, dt)
    assert not S[0].any() and not S[1].any()
    X = mg.direct_solve(eta, h, 0.5 * dt, S)
    scale = np.abs(X).max()
    assert np.abs(X[:2]).max() <= 1e-13 * scale
    assert np.abs(X[2] - X[2][:1]).max() <= 1e-13 * scale
    assert np.abs(div_c(X, h)).max() <= 1e-12 * scale / h


def _oblique_mode(n, h):
    """B_c = v_c cos(k.x) on an (4, n, n) grid, k = 2 pi (1, 2, 0) on the unit
    square, v orthogonal to the central-difference symbol cc(k) (so div_c B = 0
    to rounding) and of unit length."""
    k = 2 * np.pi * np.array([1.0, 2.0, 0.0])
    cc = np.sin(k * h) / h
    v = np.array([cc[1], -cc[0], 0.0])
    v /= np.linalg.norm(v)
    z, y, x = np.meshgrid((np.arange(4) + 0.5) * h, (np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h,
                          indexing="ij")
    B = v[:, None, None, None] * np.cos(k[0] * x + k[1] * y)[None]
    return k, v, cc, B


def _step_divergence(k, v, cc, h, eta0, dt):
    """cc . G(k) v: amplitude of the divergence one step gives the mode."""
    M = eta0 * closed.symbol(k[0], k[1], k[2], h)
    G = np.linalg.solve(np.eye(3) + 0.5 * dt * M, np.eye(3) - 0.5 * dt * M)
    return cc @ (G @ v)


@pytest.mark.parametrize("eta0", [1.0, 0.3])
def test_divergence_created_by_a_step_matches_the_symbol_and_is_second_order(eta0):
    """One step (lambda = 1/2, fixed dt) of a discretely divergence-free oblique
    mode, solved by sparse LU through the oracle's operator, creates the
    divergence -(cc . G(k) v) sin(k.x) with G the step's Fourier factor; that
    amplitude over |k| falls towards a factor 4 per halving of h."""
    dt = 2e-3
    for n in (16, 32):
        h = 1.0 / n
        k, v, cc, B = _oblique_mode(n, h)
        assert np.abs(div_c(B, h)).max() <= 1e-11
        eta = np.full(B.shape[1:], eta0)
        X = mg.direct_solve(eta, h, 0.5 * dt, ref.source(B, eta, h, dt))
        d_exact = _step_divergence(k, v, cc, h, eta0, dt)
        assert d_exact != 0
        z, y, x = np.meshgrid((np.arange(4) + 0.5) * h, (np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h,
                              indexing="ij")
        expect = -d_exact * np.sin(k[0] * x + k[1] * y)   # div_c of a cos(k.x) pattern
        assert np.abs(div_c(X, h) - expect).max() <= 1e-9 * abs(d_exact) + 1e-10
    rel = []
    for n in (16, 32, 64, 128, 256):
        h = 1.0 / n
        k, v, cc, _ = _oblique_mode(4, h)
        rel.append(abs(_step_divergence(k, v, cc, h, eta0, dt)) / np.linalg.norm(k))
    ratios = [rel[i] / rel[i + 1] for i in range(len(rel) - 1)]
    assert all(3.4 <= r <= 4.4 for r in ratios), ratios
    assert abs(ratios[-1] - 4.0) <= 0.05 and abs(ratios[-1] - 4.0) < abs(ratios[0] - 4.0), ratios
