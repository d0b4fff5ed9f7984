"""Pins of the oracle's Crank-Nicolson solve: the FFT closed form of the
discrete step, a sparse direct solve, the paper's convergence orders (section
3.1), its printed amplitude and its one-iteration residual (Fig. 6)."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import closed, mg, ref

from golden_values import paper


def test_cn_step_matches_fft_closed_form():
    """Constant eta, periodic: the oracle's V-cycle-preconditioned BiCGStab
    solution equals the exact discrete step G(k) b (FFT), 16^3, r = 3.33."""
    n = 16
    h = 1.0 / n
    B = gen.divfree(n, 1.0, seed=11)
    eta = np.ones((n, n, n))
    dt = gen.explicit_dt(h, 1.0, 20.0)
    out, hist = mg.cn_step(B, eta, h, dt, rtol=1e-13)
    ex = closed.cn_exact(B, 1.0, h, dt)
    assert hist[-1] <= 1e-13
    assert np.linalg.norm(out - ex) <= 1e-12 * np.linalg.norm(ex)


def test_config_fourier32_closed_form():
    """The 32^3 three-mode workload: oracle step vs FFT closed form."""
    cfg = gen.config_fourier32()
    h = cfg["spec"].dx0
    out, hist = mg.cn_step(cfg["B"], cfg["eta"], h, cfg["dt"], rtol=1e-13)
    ex = closed.cn_exact(cfg["B"], 1.0, h, cfg["dt"])
    assert np.linalg.norm(out - ex) <= 1e-12 * np.linalg.norm(ex)


@pytest.mark.parametrize("method", ["bicgstab", "ir"])
def test_iterative_solves_match_sparse_direct(method):
    """Variable eta (log-normal, 3 decades), 8^3: multigrid solvers vs SuperLU."""
    n, h = 8, 1.0 / 8
    eta = gen.lognormal_eta(n, 3.0, seed=12)
    B = gen.divfree(n, 2.0, seed=13)
    dt = gen.explicit_dt(h, 1.0, 50.0)
    direct, _ = mg.cn_step(B, eta, h, dt, method="direct")
    it, hist = mg.cn_step(B, eta, h, dt, method=method, rtol=1e-13, maxit=400)
    assert hist[-1] <= 1e-13
    assert np.linalg.norm(it - direct) <= 1e-11 * np.linalg.norm(direct)
    # and the direct answer satisfies L B = S
    S = ref.source(B, eta, h, dt)
    R = ref.residual(direct, S, eta, h, 0.5 * dt)
    assert np.linalg.norm(R) <= 1e-12 * np.linalg.norm(S)


def test_fmg_reduces_residual():
    n, h = 16, 1.0 / 16
    eta = gen.lognormal_eta(n, 2.0, seed=14)
    S = gen.divfree(n, 2.0, seed=15)
    lv = mg.hierarchy(eta, h, 0.5 * gen.explicit_dt(h, 1.0, 20.0))
    e = mg.fmg(lv, S, n_v=2)
    r = S - lv[0].L(e)
    assert np.linalg.norm(r) < 0.05 * np.linalg.norm(S)


def _fmg_case(n):
    h = 1.0 / n
    eta = gen.lognormal_eta(n, 3.0, seed=21)
    lam_dt = 0.5 * gen.explicit_dt(h, 1.0, 20.0)
    return mg.hierarchy(eta, h, lam_dt), gen.divfree(n, 3.0, seed=22), eta, h, lam_dt


@pytest.mark.parametrize("n", [8, 16])
def test_fmg_with_many_cycles_reaches_the_solution(n):
    """FMG iterates the residual equation on the finest level, so with enough
    V-cycles per level it returns L^{-1} r whatever its start: 2 and 3 levels,
    log-normal eta over three decades.  The result satisfies L X = S to
    rounding (L the oracle's operator, pinned on its own), and at 8^3 equals
    SuperLU's solution."""
    lv, S, eta, h, lam_dt = _fmg_case(n)
    assert len(lv) == (2 if n == 8 else 3)
    X = mg.fmg(lv, S, n_v=40)
    assert np.linalg.norm(ref.residual(X, S, eta, h, lam_dt)) <= 1e-13 * np.linalg.norm(S)
    if n == 8:
        Xd = mg.direct_solve(eta, h, lam_dt, S)
        assert np.linalg.norm(X - Xd) <= 1e-12 * np.linalg.norm(Xd)


def test_fmg_start_beats_a_vcycle_from_zero():
    """What makes it full multigrid: each level starts from the interpolated
    coarser solution, so for a smooth right-hand side one V-cycle per level
    leaves a small fraction of the error one V-cycle from zero leaves (0.14
    here; without the interpolated start the two coincide).  The exact answer
    is FMG's limit, whose residual is checked."""
    lv, S, eta, h, lam_dt = _fmg_case(16)
    X = mg.fmg(lv, S, n_v=40)
    assert np.linalg.norm(ref.residual(X, S, eta, h, lam_dt)) <= 1e-13 * np.linalg.norm(S)
    e_fmg = np.linalg.norm(mg.fmg(lv, S, n_v=1) - X)
    e_v = np.linalg.norm(mg.vcycle(lv, S) - X)
    assert e_fmg < 0.3 * e_v, (e_fmg, e_v)


def test_heat_factor_and_paper_amplitude():
    """Sinusoidal test (section 3.1): B_z = sin(k.r), k = 2 pi (1, 2, 0),
    eta = 1, box [0,1] x [0,1/2] x [0,1/4].  The z-only field evolves as the
    5-point heat equation: amplitude = g^n exactly; at t = 4e-3 it is close to
    exp(-eta |k|^2 t) = 0.454, which the paper prints as 0.45."""
    h = 1.0 / 64
    nx, ny, nz = 64, 32, 16
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    kx, ky = 2 * np.pi, 4 * np.pi
    B = np.zeros((3, nz, ny, nx))
    B[2] = np.sin(kx * x + ky * y)
    eta = np.ones((nz, ny, nx))
    dt, nsteps = 1e-3, 4
    b = B
    for _ in range(nsteps):
        b, hist = mg.cn_step(b, eta, h, dt, rtol=1e-13)
    g = closed.heat_factor(kx, ky, h, 1.0, dt) ** nsteps
    assert np.abs(b[2] - g * B[2]).max() < 1e-11
    assert np.abs(b[:2]).max() < 1e-12
    amp = g
    exact = closed.continuum_decay(kx ** 2 + ky ** 2, 1.0, 4e-3)
    assert abs(exact - 0.4540) < 1e-4
    assert abs(amp - exact) < 5e-3
    printed = paper("sinusoid_amplitude_t4e-3")
    assert round(amp, printed["digits"]) == printed["value"]


def _sinusoid_error(n_cells_per_unit, dt, t_end, lam):
    h = 1.0 / n_cells_per_unit
    nx, ny, nz = n_cells_per_unit, n_cells_per_unit // 2, n_cells_per_unit // 4
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    kx, ky = 2 * np.pi, 4 * np.pi
    B = np.zeros((3, nz, ny, nx))
    B[2] = np.sin(kx * x + ky * y)
    eta = np.ones((nz, ny, nx))
    b = B
    for _ in range(int(round(t_end / dt))):
        b, _h = mg.cn_step(b, eta, h, dt, lam=lam, rtol=1e-13)
    ex = closed.continuum_decay(kx ** 2 + ky ** 2, 1.0, t_end) * B[2]
    semi = np.exp(-t_end * ((2 / h * np.sin(kx * h / 2)) ** 2 + (2 / h * np.sin(ky * h / 2)) ** 2)) * B[2]
    return np.abs(b[2] - ex).mean(), np.abs(b[2] - semi).mean()


def test_temporal_order():
    """lambda = 1/2 is second order in dt, lambda = 1 first order (Fig. 2):
    errors against the spatially exact-in-time (semi-discrete) solution."""
    errs = {0.5: [], 1.0: []}
    dts = [1e-3, 5e-4, 2.5e-4]
    for lam in (0.5, 1.0):
        for dt in dts:
            errs[lam].append(_sinusoid_error(32, dt, 2e-3, lam)[1])
    order = paper("temporal_order")["value"]
    for lam in (0.5, 1.0):
        slope = np.log(errs[lam][0] / errs[lam][-1]) / np.log(dts[0] / dts[-1])
        assert abs(slope - order[str(lam)]) <= 0.1 * order[str(lam)], (lam, slope)


def test_spatial_order():
    """Both schemes are second order in space (Fig. 5): dt = 4e-3 (8/N)^2 ...
    scaled so the run stays small; error against exp(-eta k^2 t)."""
    errs = []
    ns = [16, 32, 64]
    for n in ns:
        dt = 2e-4 * (16 / n) ** 2
        errs.append(_sinusoid_error(n, dt, 4e-4, 0.5)[0])
    s = np.log(errs[0] / errs[-1]) / np.log(ns[-1] / ns[0])
    assert abs(s - paper("spatial_order")["value"]) <= 0.2, s


def test_one_iteration_residual_fig6():
    """Fig. 6 (section 3.1) on the unrefined sinusoid box: one iteration of
    eqs. (16)-(18) from B^n, the multigrid step being FMG with Table 1's first
    schedule (4 V-cycles, 4 + 4 sweeps), leaves max|R| below 1e-5 for
    eta dt / h^2 from 0.1 to 16.4 (N = 8 and 16, dt = 4e-3 and 1e-4, both
    lambda); lambda = 1/2 ends lower than lambda = 1, and a smaller
    eta dt / h^2 lower than a larger one, as the paper observes."""
    row = paper("table1_schedules")["value"]["FMG on AMR"]
    bound = paper("one_iteration_max_residual")["value"]
    r1 = {}
    for N in (8, 16):
        h = 1.0 / (4 * N)
        nx, ny, nz = 4 * N, 2 * N, N
        z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                              (np.arange(nx) + 0.5) * h, indexing="ij")
        B = np.zeros((3, nz, ny, nx))
        B[2] = np.sin(2 * np.pi * x + 4 * np.pi * y)
        eta = np.ones((nz, ny, nx))
        for dt in (4e-3, 1e-4):
            for lam in (0.5, 1.0):
                S = ref.source(B, eta, h, dt, lam)
                lv = mg.hierarchy(eta, h, lam * dt)
                R0 = S - lv[0].L(B)
                X = B + mg.fmg(lv, R0, n_v=row["v_cycles"], nu1=row["pre"], nu2=row["post"])
                r1[N, dt, lam] = np.abs(S - lv[0].L(X)).max()
                assert np.abs(R0).max() > 1e3 * bound
                assert r1[N, dt, lam] < bound, (N, dt, lam, r1[N, dt, lam])
    for N in (8, 16):
        assert r1[N, 4e-3, 0.5] < r1[N, 4e-3, 1.0], r1
        for lam in (0.5, 1.0):
            assert r1[N, 1e-4, lam] < r1[N, 4e-3, lam], r1
