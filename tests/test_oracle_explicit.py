"""Pins of the oracle's explicit predictor-corrector scheme (section 3.3):
the FFT closed form of the scheme for constant resistivity, second order in
time against the time-exact space-discrete solution, conservation of the
volume integral on an AMR hierarchy (flux form with refluxing), uniform
refinement = one fine level, and the paper's comparison (the lambda = 1/2
implicit solution agrees with the explicit one much better than lambda = 1)."""
import numpy as np

import ohm_inputs as gen
from oracle import amr, closed, explicit, mg, ref


def test_heun_matches_fft_closed_form():
    n, eta0 = 16, 0.7
    h = 1.0 / n
    b = gen.divfree(n, 1.0, seed=3)
    eta = np.full((n, n, n), eta0)
    dt = 0.4 * h * h / (6 * eta0)
    got = explicit.heun_steps(b, eta, h, dt, 5)
    ex = closed.heun_exact(b, eta0, h, dt, 5)
    assert np.abs(got - ex).max() <= 1e-13 * np.abs(ex).max()
    # a planted forward-Euler corrector (no trapezoidal average) is caught
    bad = b - dt * ref.div(ref.flux(b, eta, h), h)
    assert np.abs(bad - closed.heun_exact(b, eta0, h, dt, 1)).max() > 1e-6


def test_heun_second_order_in_time():
    n, eta0, T = 16, 1.0, 1e-3
    h = 1.0 / n
    b = gen.divfree(n, 1.0, seed=4)
    eta = np.full((n, n, n), eta0)
    ex = closed.semidiscrete_exact(b, eta0, h, T)
    errs = []
    for k in (16, 32, 64):
        errs.append(np.linalg.norm(explicit.heun_steps(b, eta, h, T / k, k) - ex))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_heun_amr_conserves_volume_integral():
    lev0 = gen.full_level((2, 2, 2))
    lev1 = gen.morton_order(np.array([(1, 1, 1), (2, 1, 1)], dtype=np.int32))
    spec = gen.HierSpec((2, 2, 2), 0.25, [lev0, lev1])
    comp = amr.Composite(spec)
    rng = np.random.default_rng(5)
    Bs, es = [], []
    for l in range(2):
        nx, ny, nz = spec.cells(l)
        Bs.append(rng.standard_normal((3, nz, ny, nx)))
        es.append(np.exp(rng.standard_normal((nz, ny, nx))))
    dt = 0.3 * spec.dx(1) ** 2 / (6 * max(e.max() for e in es))
    Bs = comp.average_down(Bs)
    out = explicit.heun_steps_amr(comp, Bs, es, dt, 3)

    def integral(X):
        return [sum(X[l][c][comp.leaf[l]].sum() * spec.dx(l) ** 3 for l in range(2)) for c in range(3)]

    a, z = integral(Bs), integral(out)
    mag = sum(np.abs(Bs[l]).sum() * spec.dx(l) ** 3 for l in range(2))
    assert all(abs(a[c] - z[c]) <= 1e-13 * mag for c in range(3))


def test_heun_amr_uniform_refinement_equals_single_level():
    spec0 = gen.HierSpec((1, 1, 1), 0.2, [gen.full_level((1, 1, 1))])
    spec = gen.HierSpec((1, 1, 1), 0.2, [spec0.levels[0], gen.morton_order(gen.children_of(spec0.levels[0]))])
    comp = amr.Composite(spec)
    rng = np.random.default_rng(6)
    Bf = rng.standard_normal((3, 16, 16, 16))
    ef = np.exp(rng.standard_normal((16, 16, 16)))
    dt = 0.3 * 0.1 ** 2 / (6 * ef.max())
    out = explicit.heun_steps_amr(comp, [np.zeros((3, 8, 8, 8)), Bf], [ref.restrict(ef), ef], dt, 2)
    ex = explicit.heun_steps(Bf, ef, 0.1, dt, 2)
    assert np.abs(out[1] - ex).max() <= 1e-13 * np.abs(ex).max()


def test_paper_comparison_cn_agrees_with_explicit():
    """Section 3.3 at a reduced size (32^3 on [-4, 4)^3, t = 0.2): the
    second-order implicit solution with dt = 0.1 is much closer to the explicit
    dt = 1e-3 solution than the first-order one."""
    cfg = gen.config_e8(32)
    h, T = cfg["spec"].dx0, 0.2
    Bx = explicit.heun_steps(cfg["B"], cfg["eta"], h, cfg["dt_explicit"], int(round(T / cfg["dt_explicit"])))
    Bc, Bb = cfg["B"].copy(), cfg["B"].copy()
    for _ in range(int(round(T / cfg["dt_implicit"]))):
        Bc, _ = mg.cn_step(Bc, cfg["eta"], h, cfg["dt_implicit"], rtol=1e-12)
        Bb, _ = mg.cn_step(Bb, cfg["eta"], h, cfg["dt_implicit"], lam=1.0, rtol=1e-12)
    ec = np.linalg.norm(Bc - Bx) / np.linalg.norm(Bx)
    eb = np.linalg.norm(Bb - Bx) / np.linalg.norm(Bx)
    print("lambda=1/2:", ec, "lambda=1:", eb)
    assert ec < 3e-3 and eb > 4 * ec


def test_heun_stability_limit():
    """The largest eigenvalue of eta M(k) is 8 eta / h^2 (at k = (0, pi/h, pi/h):
    there the central differences vanish and M is diagonal with 8/h^2 on the
    x component), and Heun's factor 1 - dt mu + (dt mu)^2 / 2 has modulus at
    most 1 exactly while dt mu <= 2: the scheme is stable up to dt = h^2 / (4
    eta) for constant eta.  The oracle's step on that mode, B_x = (-1)^(j+k),
    keeps its amplitude at the limit and multiplies it by 1.22 at 1.1 times it."""
    n, eta0 = 8, 0.5
    h = 1.0 / n
    k = np.linspace(0, np.pi / h, 17)
    K = np.meshgrid(k, k, k, indexing="ij")
    mu = np.linalg.eigvalsh(eta0 * closed.symbol(*K, h)).max()
    assert abs(mu - 8 * eta0 / h ** 2) <= 1e-9 * mu
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    b = np.zeros((3, n, n, n))
    b[0] = (-1.0) ** (y + z)
    eta = np.full((n, n, n), eta0)
    dt_max = h * h / (4 * eta0)
    for f, factor in ((1.0, 1.0), (1.1, 1 - 2.2 + 2.2 ** 2 / 2)):
        got = explicit.heun_steps(b, eta, h, f * dt_max, 1)
        assert np.abs(got - factor * b).max() <= 1e-12, f
    assert 1 - 2.2 + 2.2 ** 2 / 2 > 1.2
