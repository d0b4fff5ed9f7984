"""Pins of the oracle's composite AMR operator: uniform refinement reduces to a
single level, linear fields are reproduced exactly through the coarse-fine
ghosts and the refluxed faces, refluxing conserves the volume integral
(section 4), the composite solve matches a sparse direct solve, and on the
paper's half-refined box the step is second order in the cell width (Fig. 5).
The oracle's AMR multigrid (FMG over the AMR levels, Table 1) meets Fig. 6's
one-iteration residual bound on that box and converges to the composite
solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import ohm_inputs as gen
from oracle import amr, ref

from golden_values import paper


def _spec_one_patch(base_blocks=(2, 2, 2), patch=((1, 1, 1),), dx0=0.1):
    lev0 = gen.full_level(base_blocks)
    # a level-1 block at block coords P covers coarse cells 4P .. 4P+3
    lev1 = gen.morton_order(np.array(patch, dtype=np.int32))
    return gen.HierSpec(base_blocks, dx0, [lev0, lev1])


def test_uniform_refinement_equals_single_fine_level():
    spec0 = gen.HierSpec((1, 1, 1), 0.2, [gen.full_level((1, 1, 1))])
    lev1 = gen.children_of(spec0.levels[0])
    spec = gen.HierSpec((1, 1, 1), 0.2, [spec0.levels[0], gen.morton_order(lev1)])
    comp = amr.Composite(spec)
    rng = np.random.default_rng(0)
    Bf = rng.standard_normal((3, 16, 16, 16))
    ef = np.exp(rng.standard_normal((16, 16, 16)))
    Bs = [np.zeros((3, 8, 8, 8)), Bf]
    es = [ref.restrict(ef), ef]
    out = comp.apply(Bs, es, 0.37)
    ex = ref.apply(Bf, ef, 0.1, 0.37)
    assert np.abs(out[1] - ex).max() <= 1e-13 * np.abs(ex).max()
    assert not comp.leaf[0].any()


def test_linear_fields_exact_across_coarse_fine_interface():
    """Linear B and linear eta: fluxes are exact everywhere, including fine
    faces that use interpolated ghosts and coarse faces that take the mean of
    fine fluxes, so div F equals its continuum value (a constant)."""
    spec = _spec_one_patch(base_blocks=(3, 3, 3), patch=((2, 2, 2), (3, 2, 2), (2, 3, 2)), dx0=0.1)
    comp = amr.Composite(spec)
    a = np.array([[0.3, 1.2, -0.7, 0.4], [-0.2, 0.5, 0.9, -1.1], [1.0, -0.6, 0.3, 0.8]])
    g = np.array([2.0, 0.3, -0.2, 0.15])
    Bs, es = [], []
    for l in range(2):
        nx, ny, nz = spec.cells(l)
        h = spec.dx(l)
        z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                              (np.arange(nx) + 0.5) * h, indexing="ij")
        Bs.append(np.stack([a[c, 0] + a[c, 1] * x + a[c, 2] * y + a[c, 3] * z for c in range(3)]))
        es.append(g[0] + g[1] * x + g[2] * y + g[3] * z)
    D = comp.divF(Bs, es)
    # continuum: F_d[c] = eta (d_c B_d - d_d B_c) with constant gradients G[c, d] = dB_c/dx_d
    G = a[:, 1:]
    exact = np.array([sum(g[1 + d] * (G[d, c] - G[c, d]) for d in range(3)) for c in range(3)])
    # compare at leaf cells at least 3 coarse cells from the periodic seam
    for l in range(2):
        nx, ny, nz = spec.cells(l)
        m = 3 * (1 << l)
        sel = np.zeros_like(comp.leaf[l])
        sel[m:nz - m, m:ny - m, m:nx - m] = True
        sel &= comp.leaf[l]
        assert sel.sum() > 0
        for c in range(3):
            assert np.abs(D[l][c][sel] - exact[c]).max() < 1e-11, (l, c)


def test_refluxing_conserves_volume_integral():
    spec = _spec_one_patch(base_blocks=(2, 2, 2), patch=((1, 1, 1), (2, 1, 1)), dx0=0.25)
    comp = amr.Composite(spec)
    rng = np.random.default_rng(2)
    Bs, es = [], []
    for l in range(2):
        nx, ny, nz = spec.cells(l)
        Bs.append(rng.standard_normal((3, nz, ny, nx)))
        es.append(np.exp(rng.standard_normal((nz, ny, nx))))
    D = comp.divF(Bs, es)
    for c in range(3):
        tot = sum((D[l][c][comp.leaf[l]]).sum() * spec.dx(l) ** 3 for l in range(2))
        mag = sum(np.abs(D[l][c][comp.leaf[l]]).sum() * spec.dx(l) ** 3 for l in range(2))
        assert abs(tot) <= 1e-12 * mag


def test_composite_solve_matches_sparse_direct():
    """Tiny hierarchy (one 8^3 base block, one refined 8^3 fine block):
    assemble the composite matrix by unit probes and solve by SuperLU."""
    spec = gen.HierSpec((1, 1, 1), 0.125, [gen.full_level((1, 1, 1)),
                                          np.array([[1, 0, 1]], dtype=np.int32)])
    comp = amr.Composite(spec)
    rng = np.random.default_rng(3)
    etas = [np.exp(rng.standard_normal((8, 8, 8))), None]
    etas[1] = np.exp(rng.standard_normal((16, 16, 16)))
    lam_dt = 0.5 * gen.explicit_dt(spec.dx(1), float(max(e.max() for e in etas)), 30.0)
    nunk = sum(3 * int(m.sum()) for m in comp.leaf)
    zero = [np.zeros((3, 8, 8, 8)), np.zeros((3, 16, 16, 16))]
    cols = []
    for j in range(nunk):
        e = np.zeros(nunk)
        e[j] = 1.0
        cols.append(sp.csc_matrix(comp.pack(comp.apply(comp.unpack(e, zero), etas, lam_dt))[:, None]))
    A = sp.hstack(cols).tocsc()
    S = [rng.standard_normal(z.shape) for z in zero]
    x_direct = spla.spsolve(A, comp.pack(S))
    xs, hist = comp.solve(S, etas, lam_dt, rtol=1e-13)
    assert hist[-1] <= 1e-13
    x_it = comp.pack(xs)
    assert np.linalg.norm(x_it - x_direct) <= 1e-11 * np.linalg.norm(x_direct)
    # conservation as a matrix property: volume-weighted column sums of the
    # flux part vanish
    vol = comp.volumes()
    Adiv = (A - sp.identity(nunk)) / lam_dt
    colsum = np.asarray((sp.diags(vol) @ Adiv).sum(axis=0)).ravel()
    assert np.abs(colsum).max() <= 1e-11 * np.abs(Adiv).max() * vol.max()


def _half_refined(N):
    """Section 3.1's refined box: [0, 1] x [0, 1/2] x [0, 1/4] of 4 x 2 x 1
    base blocks of N^3 cells (here (N/8)^3 blocks of 8^3 each), x < 1/2
    refined once."""
    f = N // 8
    bb = (4 * f, 2 * f, f)
    lev0 = gen.full_level(bb)
    lev1 = gen.morton_order(gen.children_of(np.array([b for b in lev0 if b[0] < 2 * f], dtype=np.int32)))
    return gen.HierSpec(bb, 1.0 / (4 * N), [lev0, lev1])


def _sinusoid(spec, amp):
    """B_z = amp sin(k.r), k = 2 pi (1, 2, 0), at the cell centres of every level."""
    Bs = []
    for l in range(spec.nlevels):
        nx, ny, nz = spec.cells(l)
        h = spec.dx(l)
        z, y, x = np.meshgrid((np.arange(nz) + .5) * h, (np.arange(ny) + .5) * h, (np.arange(nx) + .5) * h,
                              indexing="ij")
        B = np.zeros((3, nz, ny, nx))
        B[2] = amp * np.sin(2 * np.pi * x + 4 * np.pi * y)
        Bs.append(B)
    return Bs


@pytest.mark.parametrize("lam", [0.5, 1.0])
def test_second_order_in_space_on_the_refined_grid(lam):
    """Fig. 5 (section 3.1): on the half-refined box both schemes are second
    order in the cell width.  One step of dt = 1e-3 at N = 8 and N = 16 against
    the same step taken with the exact spatial operator, B_z = g sin(k.r) with
    g = (1 - (1 - lam) dt eta|k|^2) / (1 + lam dt eta|k|^2): what is left is the
    spatial error alone, which falls by 2^order per halving of the cell width
    in the coarse and in the refined region separately, and the coarse region
    keeps the larger error (section 3.1, the text on Fig. 3).  The paper's own
    schedule, dt proportional to N^-2 up to t = 4e-3, is too long for the
    oracle here; with one step at fixed dt the spatial error scales as h^2
    just the same.  Piecewise-constant coarse-fine ghosts, or coarse faces that
    keep their own flux instead of the fine mean, measure an order of 1.1-1.2."""
    dt, k2 = 1e-3, 5 * (2 * np.pi) ** 2
    g = (1 - (1 - lam) * dt * k2) / (1 + lam * dt * k2)
    err = []
    for N in (8, 16):
        spec = _half_refined(N)
        comp = amr.Composite(spec)
        etas = [np.ones(spec.cells(l)[::-1]) for l in range(2)]
        B, hist = comp.cn_step(comp.average_down(_sinusoid(spec, 1.0)), etas, dt, lam=lam, rtol=1e-12)
        assert hist[-1] <= 1e-12
        ex = _sinusoid(spec, g)
        err.append([np.abs(B[l][2][comp.leaf[l]] - ex[l][2][comp.leaf[l]]).mean() for l in range(2)])
        assert np.abs(B[0][:2]).max() == 0.0 and np.abs(B[1][:2]).max() == 0.0
    order = paper("spatial_order")["value"]
    for l in range(2):
        measured = np.log2(err[0][l] / err[1][l])
        assert abs(measured - order) <= 0.3, (l, measured, err)
    assert all(e[0] > e[1] for e in err), err


def _half_refined_sinusoid(N):
    """Section 3.1's refined box with B_z = sin(2 pi x + 4 pi y), eta = 1."""
    spec = _half_refined(N)
    C = amr.Composite(spec)
    es = [np.ones(C.mask[l].shape) for l in range(2)]
    return spec, C, C.average_down(_sinusoid(spec, 1.0)), es


def _max_leaf(C, R):
    return max(np.abs(R[l][:, C.leaf[l]]).max() for l in range(C.L))


@pytest.mark.parametrize("dt", [4e-3, 1e-4])
@pytest.mark.parametrize("lam", [0.5, 1.0])
def test_amr_fmg_one_iteration_fig6(dt, lam):
    """Fig. 6 (section 3.1) on the half-refined grid: one iteration of eqs.
    (16)-(18) from B^n, the multigrid step being FMG over the AMR levels with
    Table 1's schedules (4 composite V-cycles of 4 + 4 sweeps on the refined
    level, then 2 more (MLAT-FAS row), the base grid by FMG with 2 V-cycles of
    2 + 2), takes max|R| from about 1 (dt = 4e-3) or 3e-2 (dt = 1e-4) below
    1e-5 at N = 8.  A single composite V-cycle does not (the first iteration
    then leaves the coarse-fine interface residual)."""
    tab = paper("table1_schedules")["value"]
    bound = paper("one_iteration_max_residual")["value"]
    spec, C, B0, es = _half_refined_sinusoid(8)
    S = C.source(B0, es, dt, lam)
    R0 = C.residual(B0, S, es, lam * dt)
    M = amr.AMRMultigrid(C, es, lam * dt, nu=tab["FMG on AMR"]["pre"], n_base=tab["FMG on base grid"]["v_cycles"],
                         nu_base=tab["FMG on base grid"]["pre"])
    e = M.fmg(R0, n_fmg=tab["FMG on AMR"]["v_cycles"], n_mlat=tab["MLAT-FAS on AMR"]["v_cycles"])
    X = C.average_down([B0[l] + np.where(C.leaf[l][None], e[l], 0.0) for l in range(2)])
    r0, r1 = _max_leaf(C, R0), _max_leaf(C, C.residual(X, S, es, lam * dt))
    print("max|R|", r0, "->", r1)
    assert r0 > 1e3 * bound and r1 < bound
    one = M.vcycles(R0, 1)
    X1 = C.average_down([B0[l] + np.where(C.leaf[l][None], one[l], 0.0) for l in range(2)])
    assert _max_leaf(C, C.residual(X1, S, es, lam * dt)) > 10 * bound


def test_amr_multigrid_iteration_reaches_the_composite_solution():
    """Iterating x <- x + M(S - L_comp x) with one composite V-cycle converges
    to the composite solution of the sparse-direct-checked solver, on the
    hierarchy of the composite-solve pin (variable eta, 3 decades)."""
    spec = gen.HierSpec((2, 2, 2), 1.0 / 16,
                        [gen.full_level((2, 2, 2)), np.array([[1, 1, 1], [2, 1, 1]], dtype=np.int32)])
    C = amr.Composite(spec)
    rng = np.random.default_rng(17)
    Bs = C.average_down([C.to_dense(l, rng.standard_normal((3, len(spec.levels[l]), 8, 8, 8))) for l in range(2)])
    es = [C.to_dense(l, 10 ** rng.uniform(-3, 0, (len(spec.levels[l]), 8, 8, 8))) for l in range(2)]
    es = [np.where(np.isnan(e), 1.0, e) for e in es]
    dt = gen.explicit_dt(spec.dx(1), 1.0, 40.0)
    S = C.source(Bs, es, dt)
    ex, _ = C.solve(S, es, 0.5 * dt, rtol=1e-13)
    M = amr.AMRMultigrid(C, es, 0.5 * dt, nu=2, n_base=1, nu_base=2)
    x = [b.copy() for b in Bs]
    nS = np.linalg.norm(C.pack(S))
    for it in range(60):
        R = C.residual(x, S, es, 0.5 * dt)
        if np.linalg.norm(C.pack(R)) <= 1e-12 * nS:
            break
        e = M.vcycles(R, 1)
        x = C.average_down([x[l] + np.where(C.leaf[l][None], e[l], 0.0) for l in range(2)])
    print("iterations", it)
    assert it < 60
    assert np.linalg.norm(C.pack(x) - C.pack(ex)) <= 1e-10 * np.linalg.norm(C.pack(ex))
