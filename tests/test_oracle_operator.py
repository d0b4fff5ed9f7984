"""Pins of the oracle's discrete operator (eqs. 4-11, 13, 19-23) against facts
that do not come from the oracle itself: a Fourier closed form, exactness on
polynomials against the symbolic continuum operator, the 2-D variable-
coefficient heat stencil, conservation, and dense linear algebra."""
import numpy as np
import pytest
import sympy

from oracle import closed, mg, ref


def _mode(n, h, m, v):
    nx, ny, nz = n
    k = 2 * np.pi * np.array([m[0] / (nx * h), m[1] / (ny * h), m[2] / (nz * h)])
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    return k, ph


@pytest.mark.parametrize("m", [(1, 0, 0), (1, 2, 3), (3, -1, 2), (4, 3, 5), (0, 0, 0), (2, 3, -4)])
def test_fourier_symbol(m):
    """div F of a Fourier mode equals eta M(k) v (constant eta): pins the signs,
    the component/direction indices and both difference formulas (9), (10)."""
    n, h, eta0 = (8, 6, 10), 0.37, 1.7
    rng = np.random.default_rng(abs(hash(m)) % 1000)
    v = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    k, ph = _mode(n, h, m, v)
    B = np.real(v[:, None, None, None] * ph[None])
    eta = np.full(ph.shape, eta0)
    D = ref.div(ref.flux(B, eta, h), h)
    Mv = eta0 * closed.symbol(k[0], k[1], k[2], h) @ v
    expect = np.real(Mv[:, None, None, None] * ph[None])
    scale = max(1.0, np.abs(expect).max())
    assert np.abs(D - expect).max() <= 1e-12 * scale


def _curlcurl_exact(seed):
    """Random quadratic B and linear eta; return numeric functions of the
    continuum div F = curl(eta curl B) (eqs. 3-6), by sympy."""
    x, y, z = sympy.symbols("x y z")
    rng = np.random.default_rng(seed)
    mons = [1, x, y, z, x * x, y * y, z * z, x * y, y * z, x * z]
    B = [sum(sympy.Rational(int(rng.integers(-9, 10)), 7) * mo for mo in mons) for _ in range(3)]
    g = [sympy.Rational(int(rng.integers(-3, 4)), 11) for _ in range(3)]
    eta = 2 + g[0] * x + g[1] * y + g[2] * z
    X = (x, y, z)
    curl = lambda A: [sympy.diff(A[2], y) - sympy.diff(A[1], z),
                      sympy.diff(A[0], z) - sympy.diff(A[2], x),
                      sympy.diff(A[1], x) - sympy.diff(A[0], y)]
    J = curl(B)
    out = curl([eta * J[0], eta * J[1], eta * J[2]])
    f = [sympy.lambdify(X, sympy.expand(o), "numpy") for o in out]
    fb = [sympy.lambdify(X, b, "numpy") for b in B]
    fe = sympy.lambdify(X, eta, "numpy")
    return fb, fe, f


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_on_quadratic_fields(seed):
    """For quadratic B and linear eta every difference in (9)-(11) and (8) is
    exact, so the discrete div F equals curl(eta curl B) at interior cells."""
    n, h = 10, 0.125
    fb, fe, f = _curlcurl_exact(seed)
    c = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    B = np.stack([np.broadcast_to(b(X, Y, Z), X.shape) for b in fb]).astype(float)
    eta = np.broadcast_to(fe(X, Y, Z), X.shape).astype(float)
    D = ref.div(ref.flux(B, eta, h), h)
    s = slice(2, n - 2)
    for comp in range(3):
        ex = np.broadcast_to(f[comp](X, Y, Z), X.shape)
        err = np.abs(D[comp][s, s, s] - ex[s, s, s]).max()
        assert err <= 1e-10 * max(1.0, np.abs(ex[s, s, s]).max()), (comp, err)


def test_reduces_to_2d_variable_heat_stencil():
    """B = (0, 0, Bz(x, y)) and eta(x, y): the operator is the textbook 5-point
    variable-coefficient diffusion stencil with arithmetic-mean face eta, and
    the x, y components vanish."""
    rng = np.random.default_rng(3)
    nx, ny, nz, h = 9, 7, 4, 0.3
    bz = rng.standard_normal((ny, nx))
    e2 = np.exp(rng.standard_normal((ny, nx)))
    B = np.zeros((3, nz, ny, nx))
    B[2] = bz[None]
    eta = np.broadcast_to(e2[None], (nz, ny, nx)).copy()
    D = ref.div(ref.flux(B, eta, h), h)
    ex = np.zeros_like(bz)
    for ax in (0, 1):
        ep = 0.5 * (e2 + np.roll(e2, -1, axis=ax))
        em = 0.5 * (e2 + np.roll(e2, 1, axis=ax))
        ex -= (ep * (np.roll(bz, -1, axis=ax) - bz) - em * (bz - np.roll(bz, 1, axis=ax))) / h ** 2
    assert np.abs(D[0]).max() < 1e-12 and np.abs(D[1]).max() < 1e-12
    assert np.abs(D[2] - ex[None]).max() <= 1e-12 * np.abs(ex).max()


def test_conservation_per_component():
    """Flux form: the cell sum of div F vanishes per component (periodic)."""
    rng = np.random.default_rng(4)
    B = rng.standard_normal((3, 6, 8, 10))
    eta = np.exp(2 * rng.standard_normal((6, 8, 10)))
    h = 0.2
    D = ref.div(ref.flux(B, eta, h), h)
    for c in range(3):
        assert abs(D[c].sum()) <= 1e-12 * np.abs(D[c]).sum()


def test_alpha_is_exact_diagonal():
    """alpha of (21)-(23) is the diagonal of lam dt div F (eqs. 8-13)."""
    rng = np.random.default_rng(5)
    eta = np.exp(rng.standard_normal((6, 5, 4)))
    h, lam_dt = 0.25, 0.031
    M = mg.assemble(eta, h, lam_dt)
    al = ref.alpha(eta, h, lam_dt)
    assert np.abs(M.diagonal() - (1.0 + al.ravel())).max() <= 1e-13 * (1 + al.max())


def test_symmetry_constant_vs_variable_eta():
    """Constant eta: A is symmetric; variable eta: it is not."""
    rng = np.random.default_rng(6)
    h = 0.2
    A = mg.assemble(np.full((4, 4, 6), 1.3), h, 1.0).toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    A = mg.assemble(np.exp(rng.standard_normal((4, 4, 6))), h, 1.0).toarray()
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


def test_rb_halfsweep_against_dense_algebra():
    """One red and one black half-sweep equal the dense-matrix update
    x_C += D_C^{-1} (S - L x)_C on the cells C of that colour."""
    rng = np.random.default_rng(7)
    nz, ny, nx, h, lam_dt = 6, 4, 4, 0.3, 0.05
    eta = np.exp(rng.standard_normal((nz, ny, nx)))
    B = rng.standard_normal((3, nz, ny, nx))
    S = rng.standard_normal((3, nz, ny, nx))
    L = mg.assemble(eta, h, lam_dt).toarray()
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    col = np.broadcast_to(((I + J + K) % 2)[None], B.shape).ravel()
    x = B.ravel().copy()
    for colour in (0, 1):
        r = S.ravel() - L @ x
        sel = col == colour
        x[sel] += r[sel] / np.diag(L)[sel]
        B = ref.rb_halfsweep(B, S, eta, h, lam_dt, colour)
        assert np.abs(B.ravel() - x).max() <= 1e-13 * np.abs(x).max()


def test_restrict_and_prolong_special_cases():
    rng = np.random.default_rng(8)
    f = rng.standard_normal((3, 8, 6, 4))
    c = ref.restrict(f)
    assert np.allclose(c.sum(axis=(1, 2, 3)) * 8, f.sum(axis=(1, 2, 3)), rtol=0, atol=1e-12)
    assert np.allclose(c[1, 1, 2, 0], f[1, 2:4, 4:6, 0:2].mean(), atol=1e-15)
    assert np.allclose(ref.restrict(np.full((4, 4, 4), 2.5)), 2.5)
    # prolongation reproduces constants and, away from the seam, linear fields
    assert np.allclose(ref.prolong(np.full((1, 3, 4, 5), -1.25)), -1.25, atol=1e-15)
    n = 8
    z, y, x = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    lin = 0.3 + 1.1 * x - 0.7 * y + 0.45 * z
    fine = ref.prolong(lin)
    zf, yf, xf = np.meshgrid((np.arange(2 * n) + 0.5) / 2, (np.arange(2 * n) + 0.5) / 2,
                             (np.arange(2 * n) + 0.5) / 2, indexing="ij")
    linf = 0.3 + 1.1 * xf - 0.7 * yf + 0.45 * zf
    s = slice(2, 2 * n - 2)
    assert np.abs(fine[s, s, s] - linf[s, s, s]).max() < 1e-13
    # one fine cell written out: weights 27/9/3/1 over 64 toward its side
    cc = rng.standard_normal((4, 4, 4))
    fv = ref.prolong(cc)[3, 4, 5]          # fine (I,J,K) = (5,4,3): parent (2,2,1)
    i, j, k, si, sj, sk = 2, 2, 1, 1, -1, 1
    w = {0: 0.75, 1: 0.25}
    ex = sum(w[a] * w[b] * w[g] * cc[k + g * sk, j + b * sj, i + a * si]
             for a in (0, 1) for b in (0, 1) for g in (0, 1))
    assert abs(fv - ex) < 1e-15


@pytest.mark.parametrize("r", [3.3, 16.7, 262.0])
def test_step_operator_is_bounded_below_by_one(r):
    """The whole-step bound |B - B*| <= |R| / sigma_min(L) uses sigma_min(L) >= 1.
    Constant eta: A = (L - I) / (lam dt) is symmetric positive semi-definite
    (its symbol is PSD), so every eigenvalue of L is at least 1.  Variable eta
    (3 decades): A is not symmetric and the symmetric part of A can be
    indefinite, yet the smallest singular value of L stays at 1 for every
    ratio eta_max dt / h^2 of the workloads."""
    rng = np.random.default_rng(11)
    shape, h = (4, 4, 6), 0.2
    lam_dt = r * h * h
    L = mg.assemble(np.full(shape, 1.0), h, lam_dt).toarray()
    A = (L - np.eye(len(L))) / lam_dt
    assert np.linalg.eigvalsh((A + A.T) / 2).min() >= -1e-10 * np.abs(A).max()
    assert np.linalg.eigvalsh((L + L.T) / 2).min() >= 1 - 1e-9
    eta = 10.0 ** rng.uniform(-3, 0, shape)
    L = mg.assemble(eta, h, lam_dt).toarray()
    A = (L - np.eye(len(L))) / lam_dt
    assert np.linalg.eigvalsh((A + A.T) / 2).min() < -1e-3 * np.abs(A).max()
    sv = np.linalg.svd(L, compute_uv=False)
    assert sv.min() >= 1 - 1e-9, sv.min()


def test_null_space_is_the_one_dimensional_gradients():
    """The flux divergence of eqs. (8)-(11) annihilates exactly the fields
    (f(x), g(y), h(z)) -- every flux term is a transverse difference of a
    component along its own axis or of another component, which vanish for
    such fields -- for any resistivity; with constant eta nothing else is
    annihilated: the symbol M(k) is singular only on the axis-aligned
    wavevectors, 3 n zero eigenvalues on an n^3 grid (constants included),
    while the central-difference gradient direction cc(k) of any other
    wavevector keeps the Rayleigh quotient (h^2 / 4) sum_{c != d} cc_c^2 s_d^4
    / |cc|^2 > 0 (fourth order in k: the near-null space of the step operator
    that no discrete gradient spans exactly)."""
    n, h = 8, 1.0 / 8
    rng = np.random.default_rng(5)
    eta = np.exp(rng.standard_normal((n, n, n)))
    x = np.arange(n)
    B = np.zeros((3, n, n, n))
    B[0] = rng.standard_normal(n)[None, None, :]          # f(x)
    B[1] = rng.standard_normal(n)[None, :, None]          # g(y)
    B[2] = rng.standard_normal(n)[:, None, None]          # h(z)
    assert np.abs(ref.apply(B, eta, h, 1.0) - B).max() <= 1e-13 * np.abs(B).max()
    # a field that is not of that form is not annihilated
    C = B.copy()
    C[0] += np.sin(2 * np.pi * x / n)[None, :, None]
    assert np.abs(ref.apply(C, eta, h, 1.0) - C).max() > 1e-3
    k = 2 * np.pi * np.fft.fftfreq(n, d=h)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    M = closed.symbol(KX, KY, KZ, h)
    ev = np.linalg.eigvalsh(M)
    scale = np.abs(ev).max()
    assert int((ev < 1e-12 * scale).sum()) == 3 * n
    s = np.stack([(2 / h) * np.sin(K * h / 2) for K in (KX, KY, KZ)], -1)
    cc = np.stack([np.sin(K * h) / h for K in (KX, KY, KZ)], -1)
    multi = ((KX != 0).astype(int) + (KY != 0) + (KZ != 0)) >= 2
    c2 = (cc * cc).sum(-1)
    ok = multi & (c2 > 1e-12 * scale)
    rq = np.einsum("...i,...ij,...j->...", cc, M, cc)[ok] / c2[ok]
    want = (h * h / 4) * sum(cc[..., a] ** 2 * s[..., b] ** 4 for a in range(3) for b in range(3) if a != b)[ok] / c2[ok]
    assert np.allclose(rq, want, rtol=1e-10, atol=1e-12 * scale)
    assert rq.min() > 0
