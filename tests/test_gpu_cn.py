"""Whole-step parity: one Crank-Nicolson step on the GPU against the oracle.

Bound: the GPU stops when |S - L B|_2 <= rtol |S|_2 (rtol = 1e-10, FP64
residual); with sigma_min(L) >= 1 the error is at most rtol |S|_2, and the
oracle is solved to 1e-13.  Assertion: |B_gpu - B_oracle|_2 <= 1.5 rtol |S|_2
+ 1e-12 |B_oracle|_2.  Mixed precision meets the same bound because its final
residual is FP64; its measured error is printed."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import amr, closed, mg, ref

from gpu_util import announce, blocks_to_dense, cuda, dense_to_blocks, hier, host

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _bound(S_norm, ex):
    return 1.5 * RTOL * S_norm + 1e-12 * np.linalg.norm(ex)


def _gpu_step(spec, B, eta, dt, **opts):
    import paper_1009_0798_amd as ohm
    H = hier(spec)
    ijk = spec.levels[0]
    Bt = [cuda(dense_to_blocks(B, ijk))]
    Et = [cuda(dense_to_blocks(eta, ijk)[None])]
    kw = dict(rtol=RTOL)
    kw.update(opts)
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(**kw))
    return st, stats, blocks_to_dense(host(Bt[0]), ijk, spec.cells(0))


def test_fourier32_against_closed_form():
    announce("cn fourier32 f64")
    cfg = gen.config_fourier32()
    spec, h = cfg["spec"], cfg["spec"].dx0
    st, stats, got = _gpu_step(spec, cfg["B"], cfg["eta"], cfg["dt"])
    ex = closed.cn_exact(cfg["B"], 1.0, h, cfg["dt"])
    S = ref.source(cfg["B"], cfg["eta"], h, cfg["dt"])
    print(stats, np.linalg.norm(got - ex) / np.linalg.norm(ex))
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)


@pytest.mark.parametrize("precision,outer,cycle", [(0, 1, 0), (1, 1, 0), (0, 0, 0), (0, 1, 1), (1, 0, 1)])
def test_lognormal32_against_oracle(precision, outer, cycle):
    announce(f"cn lognormal32 precision={precision} outer={outer} cycle={cycle}")
    n = 32
    spec = gen.uniform_spec(n)
    h = spec.dx0
    eta = gen.lognormal_eta(n, 4.0, seed=21)
    B = gen.divfree(n, 2.0, seed=22)
    dt = gen.explicit_dt(h, 1.0, 100.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, outer=outer, cycle=cycle, max_iters=400)
    ex, hist = mg.cn_step(B, eta, h, dt, rtol=1e-13)
    S = ref.source(B, eta, h, dt)
    err = np.linalg.norm(got - ex) / np.linalg.norm(ex)
    print("stats", stats, "rel err vs oracle", err)
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)
    # the residual the library reports is the oracle's residual of its answer
    R = ref.residual(got, S, eta, h, 0.5 * dt)
    assert np.linalg.norm(R) <= 1.01 * RTOL * np.linalg.norm(S)


@pytest.mark.parametrize("nu_pre,nu_post,nu_coarse,precision",
                         [(1, 1, 1, 0), (2, 3, 1, 0), (3, 4, 2, 1), (2, 5, 1, 0), (4, 2, 3, 1), (0, 2, 0, 0)])
def test_cycle_schedules_against_oracle(nu_pre, nu_post, nu_coarse, precision):
    """Odd and even pre/post sweep counts take different buffer paths (zero-
    guess first sweep into either buffer, correction fused into the first
    post-sweep or prolonged into the scratch buffer, dense levels likewise):
    every schedule must reach the oracle's answer."""
    announce(f"cn schedule V({nu_pre},{nu_post}) coarse {nu_coarse} precision {precision}")
    n = 32
    spec = gen.uniform_spec(n)
    h = spec.dx0
    eta = gen.lognormal_eta(n, 3.0, seed=25)
    B = gen.divfree(n, 2.0, seed=26)
    dt = gen.explicit_dt(h, 1.0, 60.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, max_iters=400, nu_pre=nu_pre,
                               nu_post=nu_post, nu_coarse=nu_coarse)
    ex, _ = mg.cn_step(B, eta, h, dt, rtol=1e-13)
    S = ref.source(B, eta, h, dt)
    print("stats", stats)
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)


@pytest.mark.parametrize("ordering,precision,cycle", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])
def test_one_iteration_equals_the_oracle_cycle(ordering, precision, cycle):
    """One iteration of eqs. (16)-(18), x1 = x0 + M(S - L x0) from x0 = b,
    against the oracle's own V(2, 2) cycle or FMG on the same hierarchy
    (32^3 -> 16^3 -> 8^3 -> 4^3, dense solve on 4^3): the GPU cycle's every
    sweep, transfer and coarse solve, red-black and four-colour.  Bound: FP64
    rounding of the correction (1e-11 of its size); mixed precision, FP32
    rounding (2e-5)."""
    import paper_1009_0798_amd as ohm
    announce(f"cn one iteration ordering={ordering} precision={precision} cycle={cycle}")
    n = 32
    spec = gen.uniform_spec(n)
    h = spec.dx0
    eta = gen.lognormal_eta(n, 3.0, seed=27)
    B = gen.divfree(n, 2.0, seed=28)
    dt = gen.explicit_dt(h, 1.0, 60.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, outer=0, cycle=cycle, n_vcycles=1,
                               nu_pre=2, nu_post=2, max_iters=1, rtol=1e-14, ordering=ordering)
    assert st == ohm._lib.OHM_ERR_NOCONV and stats[0]["iters"] == 1
    lam_dt = 0.5 * dt
    S = ref.source(B, eta, h, dt)
    levels = mg.hierarchy(eta, h, lam_dt)
    assert [lv.eta.shape[0] for lv in levels] == [32, 16, 8, 4]
    R0 = ref.residual(B, S, eta, h, lam_dt)
    e = mg.vcycle(levels, R0, 2, 2, 0, ordering) if cycle == 0 else mg.fmg(levels, R0, 1, 2, 2, ordering)
    err = np.abs(got - (B + e)).max() / np.abs(e).max()
    print("stats", stats, "max err / max correction", err)
    assert err <= (1e-11 if precision == 0 else 2e-5)
    if ordering == 1:
        # the four-colour cycle is not the red-black one
        e0 = mg.vcycle(levels, R0, 2, 2, 0, 0) if cycle == 0 else mg.fmg(levels, R0, 1, 2, 2, 0)
        assert np.abs(e - e0).max() >= 1e-4 * np.abs(e).max()


@pytest.mark.parametrize("ordering,precision", [(1, 0), (1, 1)])
def test_four_colour_step_against_oracle(ordering, precision):
    """A whole step with the four-colour smoother reaches the oracle's answer
    (BiCGStab around V(2, 2), 32^3 log-normal)."""
    announce(f"cn four-colour step precision={precision}")
    n = 32
    spec = gen.uniform_spec(n)
    h = spec.dx0
    eta = gen.lognormal_eta(n, 4.0, seed=21)
    B = gen.divfree(n, 2.0, seed=22)
    dt = gen.explicit_dt(h, 1.0, 100.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, max_iters=400, ordering=ordering)
    ex, _ = mg.cn_step(B, eta, h, dt, rtol=1e-13)
    S = ref.source(B, eta, h, dt)
    print("stats", stats, "rel err vs oracle", np.linalg.norm(got - ex) / np.linalg.norm(ex))
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)


@pytest.mark.parametrize("precision", [0, 1])
def test_backward_euler_against_oracle(precision):
    """lambda = 1 (eq. 7): S = b and L = I + dt div F."""
    announce(f"cn backward euler precision={precision}")
    n = 32
    spec = gen.uniform_spec(n)
    h = spec.dx0
    eta = gen.lognormal_eta(n, 3.0, seed=23)
    B = gen.divfree(n, 2.0, seed=24)
    dt = gen.explicit_dt(h, 1.0, 60.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, max_iters=400, lam=1.0)
    ex, _ = mg.cn_step(B, eta, h, dt, lam=1.0, rtol=1e-13)
    S = ref.source(B, eta, h, dt, 1.0)
    assert np.array_equal(S, B)
    print("stats", stats, "rel err vs oracle", np.linalg.norm(got - ex) / np.linalg.norm(ex))
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)
    R = ref.residual(got, S, eta, h, dt)
    assert np.linalg.norm(R) <= 1.01 * RTOL * np.linalg.norm(S)


def test_ragged_box_variable_eta():
    """24 x 16 x 32 box: coarsenings 12x8x16, 6x4x8, 3x2x4 (odd coarsest)."""
    announce("cn ragged box")
    spec = gen.HierSpec((3, 2, 4), 0.05, [gen.full_level((3, 2, 4))])
    nx, ny, nz = spec.cells(0)
    rng = np.random.default_rng(31)
    B = rng.standard_normal((3, nz, ny, nx))
    eta = np.exp(rng.uniform(-3, 0, (nz, ny, nx)))
    h = spec.dx0
    dt = gen.explicit_dt(h, 1.0, 30.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, max_iters=300)
    S = ref.source(B, eta, h, dt)
    ex, _ = mg.cn_step(B, eta, h, dt, rtol=1e-13, maxit=400)
    print(stats)
    assert st == 0
    assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex)


@pytest.mark.parametrize("precision,cycle", [(0, 0), (1, 0), (0, 1)])
def test_ragged_box_one_iteration_equals_the_oracle_cycle(precision, cycle):
    """One iteration of eqs. (16)-(18) on the 24 x 16 x 32 box against the
    oracle's V(2, 2) cycle or FMG on the same hierarchy: the dense levels
    12x8x16 and 6x4x8 are covered by 8^3 tiles whose last tile along an edge
    wraps around (fused sweeps, the sweep that adds the prolonged correction,
    the residual with restriction), the odd 3x2x4 coarsest grid is solved
    directly.  Bounds as for the 32^3 cycle."""
    import paper_1009_0798_amd as ohm
    announce(f"cn ragged box one iteration precision={precision} cycle={cycle}")
    spec = gen.HierSpec((3, 2, 4), 0.05, [gen.full_level((3, 2, 4))])
    nx, ny, nz = spec.cells(0)
    rng = np.random.default_rng(33)
    B = rng.standard_normal((3, nz, ny, nx))
    eta = np.exp(rng.uniform(-3, 0, (nz, ny, nx)))
    h = spec.dx0
    dt = gen.explicit_dt(h, 1.0, 30.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, outer=0, cycle=cycle, n_vcycles=1,
                               nu_pre=2, nu_post=2, nu_coarse=0, max_iters=1, rtol=1e-14)
    assert st == ohm._lib.OHM_ERR_NOCONV and stats[0]["iters"] == 1
    lam_dt = 0.5 * dt
    S = ref.source(B, eta, h, dt)
    levels = mg.hierarchy(eta, h, lam_dt)
    assert [lv.eta.shape for lv in levels] == [(32, 16, 24), (16, 8, 12), (8, 4, 6), (4, 2, 3)]
    R0 = ref.residual(B, S, eta, h, lam_dt)
    e = mg.vcycle(levels, R0, 2, 2) if cycle == 0 else mg.fmg(levels, R0, 1, 2, 2)
    err = np.abs(got - (B + e)).max() / np.abs(e).max()
    print("stats", stats, "max err / max correction", err)
    assert err <= (1e-11 if precision == 0 else 2e-5)


def test_amr_two_levels_against_oracle():
    announce("cn amr 2 levels")
    spec = gen.config_amr2(n_base=32, extra_frac=0.2, seed=4)
    C = amr.Composite(spec)
    Bb, eb = gen.amr_fields(spec, p=2.0, seed=5)
    Bs = C.average_down([C.to_dense(l, Bb[l]) for l in range(2)])
    es = [C.to_dense(l, eb[l]) for l in range(2)]
    dt = 20.0 * spec.dx(1) ** 2 / (6 * 10.0)
    import paper_1009_0798_amd as ohm
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(Bs[l], spec.levels[l])) for l in range(2)]
    Et = [cuda(dense_to_blocks(es[l], spec.levels[l])[None]) for l in range(2)]
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(rtol=RTOL, max_iters=300))
    print(stats)
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    ex, hist = C.cn_step(Bs, es, dt, rtol=1e-13)
    Ss = C.source(Bs, es, dt)
    nS = np.linalg.norm(C.pack(Ss))
    got = [blocks_to_dense(host(Bt[l]), spec.levels[l], spec.cells(l)) for l in range(2)]
    diff = np.concatenate([(got[l] - ex[l])[:, C.leaf[l]].ravel() for l in range(2)])
    exv = C.pack(ex)
    print("rel err", np.linalg.norm(diff) / np.linalg.norm(exv))
    assert np.linalg.norm(diff) <= 1.5 * RTOL * nS + 1e-12 * np.linalg.norm(exv)


@pytest.mark.parametrize("precision,ordering", [(0, 0), (1, 0), (0, 1)])
def test_amr_three_levels_corner_gap_against_oracle(precision, ordering):
    """Three levels whose finest level lacks one corner ghost: level 1 smooths
    with one launch per sweep (ghosts on every side), level 2 with half-sweeps;
    with the four-colour ordering every level takes one launch per class."""
    announce(f"cn amr 3 levels corner gap precision={precision} ordering={ordering}")
    spec = gen.config_corner_gap()
    C = amr.Composite(spec)
    Bb, eb = gen.amr_fields(spec, p=2.0, seed=7)
    L = spec.nlevels
    Bs = C.average_down([C.to_dense(l, Bb[l]) for l in range(L)])
    es = [C.to_dense(l, eb[l]) for l in range(L)]
    dt = 20.0 * spec.dx(L - 1) ** 2 / (6 * 10.0)
    import paper_1009_0798_amd as ohm
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(Bs[l], spec.levels[l])) for l in range(L)]
    Et = [cuda(dense_to_blocks(es[l], spec.levels[l])[None]) for l in range(L)]
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(rtol=RTOL, max_iters=300, precision=precision,
                                                                 ordering=ordering))
    print(stats)
    assert st == 0 and stats[0]["rel_res"] <= RTOL
    ex, _ = C.cn_step(Bs, es, dt, rtol=1e-13)
    nS = np.linalg.norm(C.pack(C.source(Bs, es, dt)))
    got = [blocks_to_dense(host(Bt[l]), spec.levels[l], spec.cells(l)) for l in range(L)]
    diff = np.concatenate([(got[l] - ex[l])[:, C.leaf[l]].ravel() for l in range(L)])
    exv = C.pack(ex)
    print("rel err", np.linalg.norm(diff) / np.linalg.norm(exv))
    assert np.linalg.norm(diff) <= 1.5 * RTOL * nS + 1e-12 * np.linalg.norm(exv)


@pytest.mark.parametrize("where", ["B", "eta"])
def test_nonfinite_input_is_reported(where):
    """A NaN in B or in the resistivity reaches the source and the initial
    residual: the step stops with OHM_ERR_NONFINITE and leaves B unchanged,
    also when it follows a clean step on the same handle (iterations and the
    copy to B are then queued before the first synchronisation)."""
    import paper_1009_0798_amd as ohm
    from paper_1009_0798_amd import _lib
    announce(f"cn non-finite input in {where}")
    n = 16
    spec = gen.uniform_spec(n)
    B = gen.divfree(n, 2.0, seed=3)
    eta = gen.lognormal_eta(n, 1.0, seed=4)
    if where == "B":
        B[1, 3, 4, 5] = np.nan
    else:
        eta[2, 5, 7] = np.nan
    H = hier(spec)
    dt = gen.explicit_dt(spec.dx0, 1.0, 50.0)
    # a clean step first, so that the failing one queues iterations (and the
    # copy to B) before its first synchronisation
    clean = [cuda(dense_to_blocks(gen.divfree(n, 2.0, seed=3), spec.levels[0]))]
    Eclean = [cuda(dense_to_blocks(gen.lognormal_eta(n, 1.0, seed=4), spec.levels[0])[None])]
    st, _ = ohm.ohm_cn_step(H, clean, Eclean, dt, ohm.default_opts())
    assert st == 0
    Bin = dense_to_blocks(B, spec.levels[0])
    Bt = [cuda(Bin)]
    Et = [cuda(dense_to_blocks(eta, spec.levels[0])[None])]
    with pytest.raises(_lib.OhmError) as err:
        ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts())
    assert err.value.status == _lib.OHM_ERR_NONFINITE
    # the failed step leaves B as it was
    assert np.array_equal(host(Bt[0]), Bin, equal_nan=True)


@pytest.mark.parametrize("lam", [0.5, 1.0])
def test_large_step_undulation_and_monotone_decay(lam):
    """Section 3.2's remark on large steps: for a high-frequency B_z(x, y)
    mode with eta dt mu = 20 one CN step multiplies it by (1 - 10)/(1 + 10) < 0
    (the mode flips sign), one backward-Euler step by 1/21 > 0 (monotone
    decay); both as the closed-form factor, to the solve tolerance."""
    import paper_1009_0798_amd as ohm
    announce(f"cn large-step mode factor lambda={lam}")
    n, h = 32, 1.0 / 32
    spec = gen.uniform_spec(n)
    z, y, x = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h,
                          indexing="ij")
    kx, ky = 2 * np.pi * 12, 2 * np.pi * 10
    B = np.zeros((3, n, n, n))
    B[2] = np.sin(kx * x + ky * y)
    mu = (2 / h * np.sin(kx * h / 2)) ** 2 + (2 / h * np.sin(ky * h / 2)) ** 2
    dt = 20.0 / mu
    g = closed.heat_factor(kx, ky, h, 1.0, dt, lam)
    assert (g < -0.8) if lam == 0.5 else (0 < g < 0.05)
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(B, spec.levels[0]))]
    Et = [cuda(dense_to_blocks(np.ones((n, n, n)), spec.levels[0])[None])]
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(lam=lam, rtol=1e-12, max_iters=300))
    assert st == 0
    got = blocks_to_dense(host(Bt[0]), spec.levels[0], spec.cells(0))
    assert np.abs(got[:2]).max() <= 1e-12
    assert np.abs(got[2] - g * B[2]).max() <= 1e-9


@pytest.mark.parametrize("ordering", [0, 1])
def test_batched_equals_alone(ordering):
    """Three problems of different sizes in one handle give the same answer as
    each solved alone (per-problem reductions in a fixed order), with either
    smoother ordering (the 24^3 problem's dense levels are not whole tiles)."""
    import paper_1009_0798_amd as ohm
    announce(f"cn batched vs alone ordering={ordering}")
    sizes = [16, 24, 32]
    probs, Bs, Es, dts = [], [], [], []
    for i, n in enumerate(sizes):
        spec = gen.uniform_spec(n)
        probs.append(spec)
        Bs.append(gen.divfree(n, 2.0, seed=40 + i))
        Es.append(gen.lognormal_eta(n, 2.0, seed=50 + i))
        dts.append(gen.explicit_dt(spec.dx0, 1.0, [20.0, 60.0, 150.0][i]))
    Hb = ohm.Hierarchy([(s.base_blocks, s.dx0, s.levels) for s in probs])
    Bcat = np.concatenate([dense_to_blocks(B, s.levels[0]) for B, s in zip(Bs, probs)], axis=1)
    Ecat = np.concatenate([dense_to_blocks(E, s.levels[0])[None] for E, s in zip(Es, probs)], axis=1)
    Bt, Et = [cuda(Bcat)], [cuda(Ecat)]
    st, stats = ohm.ohm_cn_step(Hb, Bt, Et, dts, ohm.default_opts(rtol=RTOL, ordering=ordering))
    assert st == 0
    out = host(Bt[0])
    o = 0
    for i, s in enumerate(probs):
        nb = len(s.levels[0])
        st1, stats1, alone = _gpu_step(s, Bs[i], Es[i], dts[i], ordering=ordering)
        mine = blocks_to_dense(out[:, o:o + nb], s.levels[0], s.cells(0))
        o += nb
        assert stats1[0]["iters"] == stats[i]["iters"]
        assert np.array_equal(mine, alone), i
        # and each batched answer is the oracle's (whole-step bound)
        ex, _ = mg.cn_step(Bs[i], Es[i], s.dx0, dts[i], rtol=1e-13)
        S = ref.source(Bs[i], Es[i], s.dx0, dts[i])
        assert np.linalg.norm(mine - ex) <= _bound(np.linalg.norm(S), ex), i


def test_queued_iterations_equal_step_by_step():
    """A step queues as many BiCGStab iterations as the previous step on the
    handle needed, less one, before it reads their norms; each problem is
    dropped on the device at the iteration that converges it.  A hard step
    (dt 150x explicit) followed by an easy one (dt 2x) on the same handles, a
    single problem and a batch of three, must give the easy step bit for bit
    as fresh handles do (which read after every iteration), with the same
    iteration counts."""
    import paper_1009_0798_amd as ohm
    announce("cn queued iterations vs step by step")
    sizes = [16, 24, 32]
    specs = [gen.uniform_spec(n) for n in sizes]
    Bs = [gen.divfree(n, 2.0, seed=90 + i) for i, n in enumerate(sizes)]
    Es = [gen.lognormal_eta(n, 3.0, seed=95 + i) for i, n in enumerate(sizes)]

    def run(which, multiples, H=None):
        ss = [specs[i] for i in which]
        if H is None:
            H = ohm.Hierarchy([(s.base_blocks, s.dx0, s.levels) for s in ss])
        Bt = [cuda(np.concatenate([dense_to_blocks(Bs[i], specs[i].levels[0]) for i in which], axis=1))]
        Et = [cuda(np.concatenate([dense_to_blocks(Es[i], specs[i].levels[0])[None] for i in which], axis=1))]
        dts = [gen.explicit_dt(specs[i].dx0, 1.0, m) for i, m in zip(which, multiples)]
        st, stats = ohm.ohm_cn_step(H, Bt, Et, dts, ohm.default_opts(rtol=RTOL, max_iters=300))
        assert st == 0
        return H, host(Bt[0]), stats

    for which, hard, easy in (([2], [150.0], [2.0]), ([0, 1, 2], [150.0, 60.0, 150.0], [2.0, 30.0, 1.0])):
        # hard then easy: more iterations queued than the easy step needs
        H, _, st_hard = run(which, hard)
        _, got, st_q = run(which, easy, H)
        _, ref_out, st_1 = run(which, easy)
        print(which, [s["iters"] for s in st_hard], [s["iters"] for s in st_q])
        assert max(s["iters"] for s in st_hard) - 1 > min(s["iters"] for s in st_q)   # iterations were masked
        assert [s["iters"] for s in st_q] == [s["iters"] for s in st_1]
        assert [s["rel_res"] for s in st_q] == [s["rel_res"] for s in st_1]
        assert [s["max_res"] for s in st_q] == [s["max_res"] for s in st_1]
        assert np.array_equal(got, ref_out)
        # easy then hard: fewer queued than needed, verifications queued
        # behind iterations that have not converged yet
        H, _, _ = run(which, easy)
        _, got, st_q = run(which, hard, H)
        _, ref_out, st_1 = run(which, hard)
        assert [s["iters"] for s in st_q] == [s["iters"] for s in st_1]
        assert [s["rel_res"] for s in st_q] == [s["rel_res"] for s in st_1]
        assert [s["max_res"] for s in st_q] == [s["max_res"] for s in st_1]
        assert np.array_equal(got, ref_out)


@pytest.mark.parametrize("precision", [0, 1])
def test_queued_iterations_on_amr_equal_step_by_step(precision):
    """The queued iterations, the verification formed in a scratch vector and
    the queued copy out on a 2-level AMR hierarchy (composite operator with
    refluxing and coarse-fine ghosts), FP64 and mixed: a hard step (dt 100x
    the fine level's explicit limit) then an easy one (1x) and the reverse
    on one handle equal fresh handles bit for bit, with the same counts,
    residuals and maxima."""
    import paper_1009_0798_amd as ohm
    announce(f"cn queued iterations on AMR precision={precision}")
    spec = gen.config_amr2(n_base=32, extra_frac=0.2, seed=4)
    Bb, eb = gen.amr_fields(spec, p=2.0, seed=7)
    base = spec.dx(1) ** 2 / (6 * 10.0)
    opts = ohm.default_opts(rtol=RTOL, max_iters=300, precision=precision)

    def run(mult, H=None):
        H = H if H is not None else hier(spec)
        Bt = [cuda(np.ascontiguousarray(Bb[l])) for l in range(2)]
        Et = [cuda(np.ascontiguousarray(eb[l])[None]) for l in range(2)]
        st, stats = ohm.ohm_cn_step(H, Bt, Et, mult * base, opts)
        assert st == 0
        return H, [host(b) for b in Bt], stats

    for first, second in ((100.0, 1.0), (1.0, 100.0)):
        H, _, st_a = run(first)
        _, got, st_q = run(second, H)
        _, ref_out, st_1 = run(second)
        print(first, second, st_a[0]["iters"], st_q[0]["iters"])
        for key in ("iters", "rel_res", "max_res"):
            assert st_q[0][key] == st_1[0][key], key
        for a, b in zip(got, ref_out):
            assert np.array_equal(a, b)


def test_noconv_reports_and_keeps_last_iterate():
    import paper_1009_0798_amd as ohm
    announce("cn noconv")
    n = 16
    spec = gen.uniform_spec(n)
    B = gen.divfree(n, 2.0, seed=61)
    eta = gen.lognormal_eta(n, 3.0, seed=62)
    dt = gen.explicit_dt(spec.dx0, 1.0, 100.0)
    st, stats, got = _gpu_step(spec, B, eta, dt, max_iters=1, rtol=1e-14)
    assert st == ohm._lib.OHM_ERR_NOCONV
    assert stats[0]["iters"] == 1 and stats[0]["rel_res"] > 1e-14
    S = ref.source(B, eta, spec.dx0, dt)
    R = ref.residual(got, S, eta, spec.dx0, 0.5 * dt)
    assert abs(np.linalg.norm(R) / np.linalg.norm(S) - stats[0]["rel_res"]) <= 1e-6 * stats[0]["rel_res"] + 1e-15


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_lognormal128_residual(precision):
    """128^3, eta over 4 decades, dt = 100x explicit, in the configuration the
    benchmark times (V(2, 5) cycles with one sweep below the base grid,
    captured graphs, consecutive steps on one handle): after each of two
    steps the GPU answer satisfies the oracle's own L B = S, with S built by
    the oracle from the previous step's GPU answer, to the tolerance (a
    property at any size)."""
    import paper_1009_0798_amd as ohm
    announce(f"cn 128^3 precision={precision}, two consecutive steps")
    cfg = gen.config_lognormal128()
    spec, h, dt = cfg["spec"], cfg["spec"].dx0, cfg["dt"]
    ijk = spec.levels[0]
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(cfg["B"], ijk))]
    Et = [cuda(dense_to_blocks(cfg["eta"], ijk)[None])]
    opts = ohm.default_opts(rtol=RTOL, precision=precision, max_iters=200, nu_pre=2, nu_post=5, nu_coarse=1)
    ws = ohm.Workspace()
    prev = cfg["B"]
    for step in range(2):
        st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, opts, ws)
        print(step, stats)
        assert st == 0
        got = blocks_to_dense(host(Bt[0]), ijk, spec.cells(0))
        S = ref.source(prev, cfg["eta"], h, dt)
        R = ref.residual(got, S, cfg["eta"], h, 0.5 * dt)
        assert np.linalg.norm(R) <= 1.01 * RTOL * np.linalg.norm(S), step
        prev = got


@pytest.mark.parametrize("outer", [1, 0])
def test_graph_replay_matches_eager(outer):
    """The captured outer iteration is replayed many times per step and across
    steps, with eager setup work and host synchronisation between replays:
    every step must equal the eager run bitwise."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"graph vs eager outer={outer}")
    n = 32
    spec = gen.uniform_spec(n)
    B0 = gen.divfree(n, 2.0, seed=81)
    eta = gen.lognormal_eta(n, 3.0, seed=82)
    dt = gen.explicit_dt(spec.dx0, 1.0, 50.0)
    ijk = spec.levels[0]
    res = {}
    for graph in (0, 1):
        H = hier(spec)
        Bt = [cuda(dense_to_blocks(B0, ijk))]
        Et = [cuda(dense_to_blocks(eta, ijk)[None])]
        ws = ohm.Workspace()
        outs = []
        for step in range(3):
            st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(rtol=RTOL, outer=outer, graph=graph,
                                                                       max_iters=300), ws)
            assert st == 0
            torch.cuda.synchronize()
            outs.append(Bt[0].cpu().numpy().copy())
        res[graph] = outs
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_coarse_inverse_cache_follows_eta_and_dt():
    """The coarsest-grid inverse kept in the handle is rebuilt when the
    resistivity changes in place or dt changes: results equal a fresh handle."""
    import torch
    import paper_1009_0798_amd as ohm
    announce("coarse inverse cache")
    n = 16
    spec = gen.uniform_spec(n)
    ijk = spec.levels[0]
    B0 = gen.divfree(n, 2.0, seed=91)
    e1 = gen.lognormal_eta(n, 3.0, seed=92)
    e2 = gen.lognormal_eta(n, 3.0, seed=93)
    dt1 = gen.explicit_dt(spec.dx0, 1.0, 40.0)
    dt2 = 2.5 * dt1
    H = hier(spec)
    Et = [cuda(dense_to_blocks(e1, ijk)[None])]
    ws = ohm.Workspace()
    opts = ohm.default_opts(rtol=RTOL)
    for eta, dt in ((e1, dt1), (e2, dt1), (e2, dt2)):
        Et[0].copy_(cuda(dense_to_blocks(eta, ijk)[None]))
        Bt = [cuda(dense_to_blocks(B0, ijk))]
        st, _ = ohm.ohm_cn_step(H, Bt, Et, dt, opts, ws)
        st2, _, fresh = _gpu_step(spec, B0, eta, dt)
        assert st == 0 and st2 == 0
        got = blocks_to_dense(host(Bt[0]), ijk, spec.cells(0))
        assert np.array_equal(got, fresh)


def test_degenerate_inputs():
    """B = 0: S = 0, the step returns zeros at once (relative residual 0, not
    0/0).  eta = 0 everywhere: L = I and S = b, the initial residual is exactly
    zero and B comes back bit for bit.  Zero smoothing sweeps leave B alone."""
    import torch
    import paper_1009_0798_amd as ohm
    announce("cn degenerate inputs")
    n = 16
    spec = gen.uniform_spec(n)
    eta = gen.lognormal_eta(n, 2.0, seed=71)
    dt = gen.explicit_dt(spec.dx0, 1.0, 50.0)
    st, stats, got = _gpu_step(spec, np.zeros((3, n, n, n)), eta, dt)
    assert st == 0 and stats[0]["iters"] == 0 and stats[0]["rel_res"] == 0.0
    assert not got.any()
    B = gen.divfree(n, 2.0, seed=72)
    for precision in (0, 1):
        st, stats, got = _gpu_step(spec, B, np.zeros((n, n, n)), dt, precision=precision)
        assert st == 0 and stats[0]["iters"] == 0 and stats[0]["rel_res"] == 0.0
        assert np.array_equal(got, B)
    H = hier(spec)
    ijk = spec.levels[0]
    Bt = cuda(dense_to_blocks(B, ijk))
    Et = cuda(dense_to_blocks(eta, ijk)[None])
    St = cuda(dense_to_blocks(ref.source(B, eta, spec.dx0, dt), ijk))
    before = Bt.clone()
    for ordering in (0, 1):
        ohm.ohm_smooth(H, 0, Bt, St, Et, 0.5 * dt, 0, torch.empty_like(Bt), ordering=ordering)
        assert torch.equal(Bt, before)


def _row_exchanges(A):
    """Row exchanges that Gauss-Jordan elimination with partial pivoting makes
    on A (a strictly larger entry below the diagonal is taken as pivot)."""
    A = A.copy()
    n, cnt = A.shape[0], 0
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if abs(A[p, k]) > abs(A[k, k]):
            cnt += 1
            A[[k, p]] = A[[p, k]]
        A[k] /= A[k, k]
        for r in range(n):
            if r != k:
                A[r] -= A[r, k] * A[k]
    return cnt


@pytest.mark.parametrize("precision", [0, 1])
def test_coarsest_solve_with_row_exchanges(precision):
    """The dense coarsest solve pivots.  A 16^3 box whose resistivity is
    constant on 4^3-cell cubes, with values spread over 4 decades, gives the
    4^3 coarsest grid exactly those values (means of equal children); at
    eta dt / h^2 = 100 on that grid its operator needs row exchanges (checked
    here on the oracle's assembled matrix).  One iteration of eqs. (16)-(18)
    with V(2, 2) must equal the oracle's cycle, whose coarsest solve is an
    exact inverse."""
    import paper_1009_0798_amd as ohm
    announce(f"cn coarsest solve with row exchanges precision={precision}")
    n = 16
    spec = gen.uniform_spec(n)
    h = spec.dx0
    rng = np.random.default_rng(2024)
    ec = 10.0 ** rng.uniform(-4.0, 0.0, (4, 4, 4))
    eta = np.repeat(np.repeat(np.repeat(ec, 4, axis=0), 4, axis=1), 4, axis=2)
    hc = 4 * h
    lam_dt = 100.0 * hc * hc / ec.max()
    dt = 2.0 * lam_dt
    levels = mg.hierarchy(eta, h, lam_dt)
    assert [lv.eta.shape[0] for lv in levels] == [16, 8, 4]
    assert np.allclose(levels[-1].eta, ec, rtol=1e-14, atol=0)
    assert _row_exchanges(mg.assemble(levels[-1].eta, hc, lam_dt).toarray()) > 0
    B = gen.divfree(n, 2.0, seed=2025)
    st, stats, got = _gpu_step(spec, B, eta, dt, precision=precision, outer=0, cycle=0, n_vcycles=1,
                               nu_pre=2, nu_post=2, nu_coarse=0, max_iters=1, rtol=1e-14)
    assert st == ohm._lib.OHM_ERR_NOCONV and stats[0]["iters"] == 1
    S = ref.source(B, eta, h, dt)
    R0 = ref.residual(B, S, eta, h, lam_dt)
    e = mg.vcycle(levels, R0, 2, 2)
    err = np.abs(got - (B + e)).max() / np.abs(e).max()
    print("stats", stats, "max err / max correction", err)
    assert err <= (1e-11 if precision == 0 else 2e-5)


@pytest.mark.parametrize("fmg,precision", [(1, 0), (1, 1), (0, 0)])
def test_amr_multigrid_one_iteration_equals_the_oracle(fmg, precision):
    """One iteration of eqs. (16)-(18) on the three-level hierarchy (dense-core
    eta over four decades) with the multigrid over the AMR levels: FMG over
    the levels with 2 composite V-cycles per stage and 1 more at the finest
    (fmg = 1), or 3 composite V-cycles (fmg = 0); 3 + 3 sweeps on the AMR
    levels, the base grid by FMG with 1 V-cycle of 2 + 2.  The GPU iterate
    equals the oracle's AMR multigrid (every sweep, transfer, refluxed
    coarse-fine update and base solve) to FP64 rounding of the correction, or
    FP32 rounding in mixed precision."""
    import paper_1009_0798_amd as ohm
    announce(f"cn amr multigrid one iteration fmg={fmg} precision={precision}")
    spec = gen.config_corner_gap()
    C = amr.Composite(spec)
    L = spec.nlevels
    Bb, eb = gen.amr_fields_fourier(spec, seed=29)
    Bs = C.average_down([C.to_dense(l, Bb[l]) for l in range(L)])
    es = [C.to_dense(l, eb[l]) for l in range(L)]
    dt = 20.0 * spec.dx(L - 1) ** 2 / (6 * 10.0)
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(Bs[l], spec.levels[l])) for l in range(L)]
    Et = [cuda(dense_to_blocks(es[l], spec.levels[l])[None]) for l in range(L)]
    opts = dict(outer=0, max_iters=1, rtol=1e-14, precision=precision, amr_fmg=fmg,
                amr_vcycles=2 if fmg else 3, amr_mlat=1 if fmg else 0, nu_amr=3, cycle=1, n_vcycles=1,
                nu_pre=2, nu_post=2, nu_coarse=0)
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, ohm.default_opts(**opts))
    assert st == ohm._lib.OHM_ERR_NOCONV and stats[0]["iters"] == 1
    got = [blocks_to_dense(host(Bt[l]), spec.levels[l], spec.cells(l)) for l in range(L)]
    lam_dt = 0.5 * dt
    S = C.source(Bs, es, dt)
    R0 = C.residual(Bs, S, es, lam_dt)
    M = amr.AMRMultigrid(C, es, lam_dt, nu=3, n_base=1, nu_base=2)
    e = M.fmg(R0, n_fmg=2, n_mlat=1) if fmg else M.vcycles(R0, 3)
    X = C.average_down([Bs[l] + np.where(C.leaf[l][None], e[l], 0.0) for l in range(L)])
    emax = max(np.abs(e[l][:, C.leaf[l]]).max() for l in range(L))
    err = max(np.abs(got[l][:, C.leaf[l]] - X[l][:, C.leaf[l]]).max() for l in range(L))
    r1 = C.residual(X, S, es, lam_dt)
    print("stats", stats, "max err / max correction", err / emax,
          "oracle max|R|", max(np.abs(R0[l]).max() for l in range(L)), "->", max(np.abs(r1[l]).max() for l in range(L)))
    assert err <= (1e-11 if precision == 0 else 2e-5) * emax


def test_tuned_schedule_converges_to_the_oracle():
    """The autotuner (quick table: BiCGStab around V-cycles, every pre/post
    and coarse sweep count, mixed precision) on a three-problem batch picks a
    schedule that converges, and a step with it meets the whole-step bound
    against the oracle for every problem."""
    import paper_1009_0798_amd as ohm
    from paper_1009_0798_amd import tune
    announce("tuner: chosen schedule against the oracle")
    sizes, ms = [16, 24, 32], [20.0, 80.0, 200.0]
    specs, Bs, Es, dts = [], [], [], []
    for i, n in enumerate(sizes):
        s = gen.uniform_spec(n)
        specs.append(s)
        Bs.append(gen.divfree(n, 2.0, seed=140 + i))
        Es.append(gen.lognormal_eta(n, 2.0, seed=150 + i))
        dts.append(gen.explicit_dt(s.dx0, 1.0, ms[i]))
    H = ohm.Hierarchy([(s.base_blocks, s.dx0, s.levels) for s in specs])
    B0 = cuda(np.concatenate([dense_to_blocks(B, s.levels[0]) for B, s in zip(Bs, specs)], axis=1))
    E = cuda(np.concatenate([dense_to_blocks(e, s.levels[0])[None] for e, s in zip(Es, specs)], axis=1))
    best, table = tune.tune(H, [B0], [E], dts, finest_dx=min(s.dx0 for s in specs), precisions=(1,),
                            use_cache=False, quick=True)
    print("best", best, "of", len(table))
    assert sum(1 for _, t, _ in table if t is not None) >= len(table) // 2
    Bt = [B0.clone()]
    st, stats = ohm.ohm_cn_step(H, Bt, [E], dts, ohm.default_opts(rtol=RTOL, max_iters=200, **best))
    assert st == 0
    out = host(Bt[0])
    o = 0
    for i, s in enumerate(specs):
        nb = len(s.levels[0])
        got = blocks_to_dense(out[:, o:o + nb], s.levels[0], s.cells(0))
        o += nb
        ex, _ = mg.cn_step(Bs[i], Es[i], s.dx0, dts[i], rtol=1e-13)
        S = ref.source(Bs[i], Es[i], s.dx0, dts[i])
        assert np.linalg.norm(got - ex) <= _bound(np.linalg.norm(S), ex), i
