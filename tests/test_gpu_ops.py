"""Per-call parity of the HIP building blocks against the FP64 oracle, through
the C ABI: operator apply, residual and norms, red-black smoother, restriction,
prolongation (block and dense levels), coarse-fine ghosts and refluxing.

Tolerance (FP64): every output is a sum of at most ~40 rounded products of
magnitude <= Bmax (1 + 16 |coef| eta_max / h^2); the bound is 5e-14 times that
scale.  FP32: inputs are rounded to FP32 first and the oracle runs on the
rounded values; bound 2e-5 times the same scale."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import amr, ref

from gpu_util import announce, blocks_to_dense, cuda, dense_to_blocks, hier, host

pytestmark = pytest.mark.gpu


def _scale(B, eta, coef, h):
    return np.abs(B).max() * (1.0 + 16.0 * abs(coef) * eta.max() / h ** 2)


def _setup_uniform(bb=(3, 2, 4), seed=0):
    spec = gen.HierSpec(bb, 0.05, [gen.full_level(bb)])
    nx, ny, nz = spec.cells(0)
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((3, nz, ny, nx))
    S = rng.standard_normal((3, nz, ny, nx))
    eta = np.exp(np.log(10.0) * 1.5 * rng.uniform(-1, 1, (nz, ny, nx)))
    h = spec.dx0
    lam_dt = 10.0 * h * h / eta.max()
    return spec, B, S, eta, h, lam_dt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_keeps_two_coordinate_fields(dtype):
    """B = (0, 0, B_z(x, y)) with eta(x, y): every z-plane of the result is the
    same, bit for bit (so d/dz of it is exactly zero), and the x and y
    components vanish to rounding.  They are not exact zeros: the kernel forms
    the +face and -face terms of a component in one expression, which the
    compiler contracts into a fused multiply-add, so the two equal products are
    rounded differently."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"two-coordinate field apply {dtype}")
    bb = (3, 2, 4)
    spec = gen.HierSpec(bb, 0.05, [gen.full_level(bb)])
    nx, ny, nz = spec.cells(0)
    rng = np.random.default_rng(17)
    B = np.zeros((3, nz, ny, nx))
    B[2] = rng.standard_normal((1, ny, nx))
    eta = np.broadcast_to(np.exp(rng.uniform(-1, 1, (1, ny, nx))), (nz, ny, nx))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ijk = spec.levels[0]
    H = hier(spec)
    Bt, Et = cuda(dense_to_blocks(B, ijk), tdt), cuda(dense_to_blocks(np.ascontiguousarray(eta), ijk)[None], tdt)
    out = torch.empty_like(Bt)
    coef = 0.37 * spec.dx0 ** 2
    ohm.ohm_apply(H, 0, Bt, Et, coef, out)
    got = blocks_to_dense(host(out), ijk, spec.cells(0))
    scale = _scale(B, eta, coef, spec.dx0)
    eps = 4 * float(torch.finfo(tdt).eps)
    assert all(np.array_equal(got[:, k], got[:, 0]) for k in range(nz))
    assert np.abs(got[:2]).max() <= eps * scale
    assert np.abs(got[2]).max() > 0.1 * np.abs(B[2]).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_uniform_apply_residual_smooth(dtype):
    import torch
    announce(f"uniform apply/residual/smooth {dtype}")
    spec, B, S, eta, h, lam_dt = _setup_uniform()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        B, S, eta = (x.astype(np.float32).astype(np.float64) for x in (B, S, eta))
    tol = 5e-14 if dtype == "f64" else 2e-5
    ijk = spec.levels[0]
    H = hier(spec)
    Bt, St, Et = cuda(dense_to_blocks(B, ijk), tdt), cuda(dense_to_blocks(S, ijk), tdt), cuda(dense_to_blocks(eta, ijk)[None], tdt)
    import paper_1009_0798_amd as ohm
    out = torch.empty_like(Bt)
    scale = _scale(B, eta, lam_dt, h)
    # apply
    ohm.ohm_apply(H, 0, Bt, Et, lam_dt, out)
    got = blocks_to_dense(host(out), ijk, spec.cells(0))
    ex = ref.apply(B, eta, h, lam_dt)
    assert np.abs(got - ex).max() <= tol * scale
    # residual with norms
    R = torch.empty_like(Bt)
    nrm = ohm.ohm_residual(H, 0, Bt, St, Et, lam_dt, R=R, norms=True)
    exR = ref.residual(B, S, eta, h, lam_dt)
    gotR = blocks_to_dense(host(R), ijk, spec.cells(0))
    assert np.abs(gotR - exR).max() <= tol * scale
    for c in range(3):
        assert abs(nrm[0, c, 0] - (exR[c] ** 2).sum()) <= 1e-9 * (exR[c] ** 2).sum() + tol * scale ** 2
        assert abs(nrm[0, c, 1] - np.abs(exR[c]).max()) <= tol * scale
    # smoother: 1 and 2 sweeps
    for ns in (1, 2):
        Bs = Bt.clone()
        tmp = torch.empty_like(Bt)
        ohm.ohm_smooth(H, 0, Bs, St, Et, lam_dt, ns, tmp)
        gotS = blocks_to_dense(host(Bs), ijk, spec.cells(0))
        exS = ref.smooth(B, S, eta, h, lam_dt, ns)
        assert np.abs(gotS - exS).max() <= 4 * ns * tol * scale, ns
        # four colour classes, one launch each
        Bs = Bt.clone()
        ohm.ohm_smooth(H, 0, Bs, St, Et, lam_dt, ns, tmp, ordering=1)
        gotS = blocks_to_dense(host(Bs), ijk, spec.cells(0))
        exS = ref.smooth(B, S, eta, h, lam_dt, ns, ordering=1)
        assert np.abs(gotS - exS).max() <= 8 * ns * tol * scale, ns


@pytest.mark.parametrize("dtype,bb", [("f64", (3, 2, 4)), ("f32", (3, 2, 4)), ("f64", (4, 4, 2)), ("f32", (4, 4, 2))])
def test_dense_levels_and_transfers(dtype, bb):
    """Restriction level 0 -> -1 -> -2, prolongation back, and the stencil
    calls on the dense levels.  Box 24 x 16 x 32: coarsenings 12x8x16 and
    6x4x8 (fused sweeps on 8^3 tiles, the last tile along an edge wrapping
    around) and 3x2x4 (odd: two half-sweeps); box 32 x 32 x 16: level -1 is
    16x16x8, a whole number of 8^3 tiles."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"dense levels {dtype} {bb}")
    spec, B, S, eta, h, lam_dt = _setup_uniform(bb=bb, seed=1)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        B, S, eta = (x.astype(np.float32).astype(np.float64) for x in (B, S, eta))
    tol = 5e-14 if dtype == "f64" else 2e-5
    ijk = spec.levels[0]
    H = hier(spec)
    n0 = spec.cells(0)
    assert H.problem_info(0, -1)[1] == tuple(v // 2 for v in n0)
    if bb == (3, 2, 4):
        assert H.min_level == -3 and H.problem_info(0, -3)[1] == (3, 2, 4)
    Bt = cuda(dense_to_blocks(B, ijk), tdt)
    c1 = H.field(-1, 3, tdt)
    ohm.ohm_restrict(H, 0, Bt, c1)
    ex1 = ref.restrict(B)
    assert np.abs(host(c1).reshape(ex1.shape) - ex1).max() <= tol * np.abs(B).max()
    c2 = H.field(-2, 3, tdt)
    ohm.ohm_restrict(H, -1, c1, c2)
    ex2 = ref.restrict(ex1)
    assert np.abs(host(c2).reshape(ex2.shape) - ex2).max() <= tol * np.abs(B).max()
    # prolongation -2 -> -1 (accumulate) and -1 -> 0 (overwrite)
    f1 = c1.clone()
    ohm.ohm_prolong(H, -2, c2, f1, accumulate=True)
    assert np.abs(host(f1).reshape(ex1.shape) - ref.prolong(ex2, ex1)).max() <= tol * np.abs(B).max()
    f0 = torch.empty_like(Bt)
    ohm.ohm_prolong(H, -1, c1, f0, accumulate=False)
    got = blocks_to_dense(host(f0), ijk, spec.cells(0))
    assert np.abs(got - ref.prolong(ex1)).max() <= tol * np.abs(B).max()
    # stencil calls on dense level -1 with its own resistivity and spacing
    e1 = ref.restrict(eta)
    S1 = ref.restrict(S)
    h1 = 2 * h
    et1 = cuda(e1.reshape(1, -1), tdt)
    St1 = cuda(S1.reshape(3, -1), tdt)
    out = H.field(-1, 3, tdt)
    ohm.ohm_apply(H, -1, c1, et1, lam_dt, out)
    scale = _scale(ex1, e1, lam_dt, h1)
    assert np.abs(host(out).reshape(ex1.shape) - ref.apply(ex1, e1, h1, lam_dt)).max() <= tol * scale
    ohm.ohm_residual(H, -1, c1, St1, et1, lam_dt, R=out)
    assert np.abs(host(out).reshape(ex1.shape) - ref.residual(ex1, S1, e1, h1, lam_dt)).max() <= tol * scale
    for ns in (1, 2, 3):
        Bs = c1.clone()
        ohm.ohm_smooth(H, -1, Bs, St1, et1, lam_dt, ns, torch.empty_like(c1))
        ex = ref.smooth(ex1, S1, e1, h1, lam_dt, ns)
        assert np.abs(host(Bs).reshape(ex1.shape) - ex).max() <= 8 * ns * tol * scale, ns
    if bb == (3, 2, 4):
        # level -2 (6 x 4 x 8): one 8^3 tile that wraps around in x and y
        e2, S2, h2 = ref.restrict(e1), ref.restrict(S1), 2 * h1
        et2, St2 = cuda(e2.reshape(1, -1), tdt), cuda(S2.reshape(3, -1), tdt)
        scale2 = _scale(ex2, e2, lam_dt, h2)
        for ns in (1, 2):
            Bs = c2.clone()
            ohm.ohm_smooth(H, -2, Bs, St2, et2, lam_dt, ns, torch.empty_like(c2))
            ex = ref.smooth(ex2, S2, e2, h2, lam_dt, ns)
            assert np.abs(host(Bs).reshape(ex2.shape) - ex).max() <= 8 * ns * tol * scale2, ns
    for ns in (1, 2):
        Bs = c1.clone()
        ohm.ohm_smooth(H, -1, Bs, St1, et1, lam_dt, ns, torch.empty_like(c1), ordering=1)
        ex = ref.smooth(ex1, S1, e1, h1, lam_dt, ns, ordering=1)
        assert np.abs(host(Bs).reshape(ex1.shape) - ex).max() <= 8 * ns * tol * scale, ns
    with pytest.raises(RuntimeError, match="ordering"):
        ohm.ohm_smooth(H, -1, c1.clone(), St1, et1, lam_dt, 1, torch.empty_like(c1), ordering=2)


def _amr_spec(three=False):
    bb = (4, 4, 4)
    lev0 = gen.full_level(bb)
    if not three:
        lev1 = gen.morton_order(gen.children_of(np.array([[1, 1, 1], [2, 1, 1], [1, 2, 1], [3, 3, 0]], dtype=np.int32)))
        return gen.HierSpec(bb, 1.0 / 32, [lev0, lev1])
    base = np.array([[i, j, k] for k in (1, 2) for j in (1, 2) for i in (1, 2)], dtype=np.int32)
    lev1 = gen.morton_order(gen.children_of(base))
    lev2 = gen.morton_order(gen.children_of(np.array([[3, 3, 3], [4, 3, 3]], dtype=np.int32)))
    return gen.HierSpec(bb, 1.0 / 32, [lev0, lev1, lev2])


def _amr_fields(spec, seed):
    rng = np.random.default_rng(seed)
    Bs, es = [], []
    for l in range(spec.nlevels):
        nx, ny, nz = spec.cells(l)
        Bs.append(rng.standard_normal((3, nz, ny, nx)))
        es.append(np.exp(rng.uniform(-2, 2, (nz, ny, nx))))
    return Bs, es


@pytest.mark.parametrize("nsweeps,ordering", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_smoother_with_ghosts(nsweeps, ordering):
    """Smoothing on AMR levels with ghost blocks held fixed.  Level 1 of this
    hierarchy has ghosts on faces, edges and corners (one launch per
    red-black sweep); level 2 lacks one corner ghost (two half-sweep launches
    per sweep); the four-colour ordering takes four class launches."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"smoother with ghosts nsweeps={nsweeps} ordering={ordering}")
    spec = gen.config_corner_gap()
    C = amr.Composite(spec)
    Bs, es = _amr_fields(spec, 12)
    Bs = C.average_down(Bs)
    H = hier(spec)
    Bt = [cuda(dense_to_blocks(Bs[l], spec.levels[l])) for l in range(3)]
    Et = [cuda(dense_to_blocks(es[l], spec.levels[l])[None]) for l in range(3)]
    Bfull = C.fill_ghosts(Bs)
    efull = C.fill_ghosts(es)
    coef = 0.7 * spec.dx(2) ** 2
    for l in (1, 2):
        g = H.ghost(l, 3)
        ohm.ohm_fill_ghosts(H, l, Bt[l - 1], g)
        ge = H.ghost(l, 1)
        ohm.ohm_fill_ghosts(H, l, Et[l - 1], ge)
        h = spec.dx(l)
        S = np.random.default_rng(20 + l).standard_normal(Bs[l].shape)
        St = cuda(dense_to_blocks(S, spec.levels[l]))
        Bsm = Bt[l].clone()
        ohm.ohm_smooth(H, l, Bsm, St, Et[l], coef, nsweeps, torch.empty_like(Bsm), B_ghost=g, eta_ghost=ge,
                       ordering=ordering)
        got = blocks_to_dense(host(Bsm), spec.levels[l], spec.cells(l))
        m = C.mask[l]
        x = Bfull[l].copy()
        ghost_vals = x.copy()
        classes = ref.colour_classes(efull[l].shape, ordering)
        for _ in range(nsweeps):
            for colour in range(2 if ordering == 0 else 4):
                x = ref.class_update(x, S, efull[l], h, coef, classes, colour)
                x = np.where(m[None], x, ghost_vals)
        scale = _scale(Bfull[l][:, m], efull[l], coef, h)
        err = float(np.abs(got[:, m] - x[:, m]).max())
        assert err <= 5e-13 * scale, (l, err, scale)


@pytest.mark.parametrize("three", [False, True])
def test_amr_ghosts_apply_reflux_transfers(three):
    """Level applies with coarse-fine ghosts, refluxed composite apply on the
    coarser levels, average-down restriction and prolongation, against the
    oracle's composite operator."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"amr parity three_levels={three}")
    spec = _amr_spec(three)
    C = amr.Composite(spec)
    Bs, es = _amr_fields(spec, 3 + three)
    Bs = C.average_down(Bs)
    H = hier(spec)
    L = spec.nlevels
    Bt = [cuda(dense_to_blocks(Bs[l], spec.levels[l])) for l in range(L)]
    Et = [cuda(dense_to_blocks(es[l], spec.levels[l])[None]) for l in range(L)]
    coef = 0.7 * spec.dx(L - 1) ** 2
    # restriction l -> l-1 reproduces the average-down of the oracle
    for l in range(L - 1, 0, -1):
        tgt = torch.randn_like(Bt[l - 1])
        tgt_host_before = host(tgt)
        ohm.ohm_restrict(H, l, Bt[l], tgt)
        got = blocks_to_dense(host(tgt), spec.levels[l - 1], spec.cells(l - 1))
        ex = blocks_to_dense(tgt_host_before, spec.levels[l - 1], spec.cells(l - 1))
        r = ref.restrict(np.where(C.mask[l], Bs[l], 0.0))
        ex = np.where(C.covered[l - 1], r, ex)
        m = C.mask[l - 1]
        err = float(np.abs(got[:, m] - ex[:, m]).max())
        assert err <= 1e-14 * float(np.abs(ex[:, m]).max()), ("restrict", l, err)
    # ghosts
    Bg, Eg = [None], [None]
    for l in range(1, L):
        g = H.ghost(l, 3)
        ohm.ohm_fill_ghosts(H, l, Bt[l - 1], g)
        ge = H.ghost(l, 1)
        ohm.ohm_fill_ghosts(H, l, Et[l - 1], ge)
        Bg.append(g)
        Eg.append(ge)
    Bfull = C.fill_ghosts(Bs)
    efull = C.fill_ghosts(es)
    D = C.divF(Bs, es)      # composite, refluxed
    for l in range(L):
        out = torch.empty_like(Bt[l])
        ohm.ohm_apply(H, l, Bt[l], Et[l], coef, out, B_ghost=Bg[l], eta_ghost=Eg[l])
        h = spec.dx(l)
        scale = _scale(Bfull[l][:, C.mask[l]], efull[l], coef, h)
        got = blocks_to_dense(host(out), spec.levels[l], spec.cells(l))
        # plain level apply (ghosts from the coarser level) at every level cell
        lvl = ref.apply(Bfull[l], efull[l], h, coef)
        m = C.mask[l]
        assert np.abs(got[:, m] - lvl[:, m]).max() <= 5e-14 * scale, ("level apply", l)
        if l + 1 < L:
            ohm.ohm_reflux(H, l, Bt[l], Et[l], Bt[l + 1], Et[l + 1], coef, out, B_fine_ghost=Bg[l + 1],
                           eta_fine_ghost=Eg[l + 1], zero_covered=True)
            got = blocks_to_dense(host(out), spec.levels[l], spec.cells(l))
            comp = Bs[l] + coef * D[l]
            leaf = C.leaf[l]
            assert np.abs(got[:, leaf] - comp[:, leaf]).max() <= 5e-14 * scale, ("composite", l)
            assert np.abs(got[:, C.covered[l] & m]).max() == 0.0
    # prolongation l-1 -> l onto the level blocks
    for l in range(1, L):
        out = torch.zeros_like(Bt[l])
        ohm.ohm_prolong(H, l - 1, Bt[l - 1], out, accumulate=False)
        got = blocks_to_dense(host(out), spec.levels[l], spec.cells(l))
        ex = ref.prolong(Bfull[l - 1])
        m = C.mask[l]
        assert np.abs(got[:, m] - ex[:, m]).max() <= 1e-14 * np.abs(ex).max()
    # smoother on the finest level with fixed ghosts
    l = L - 1
    h = spec.dx(l)
    S = np.random.default_rng(9).standard_normal(Bs[l].shape)
    St = cuda(dense_to_blocks(S, spec.levels[l]))
    Bsm = Bt[l].clone()
    ohm.ohm_smooth(H, l, Bsm, St, Et[l], coef, 1, torch.empty_like(Bsm), B_ghost=Bg[l], eta_ghost=Eg[l])
    got = blocks_to_dense(host(Bsm), spec.levels[l], spec.cells(l))
    x = Bfull[l].copy()
    ghost_vals = x.copy()
    for colour in (0, 1):
        x = ref.rb_halfsweep(x, S, efull[l], h, coef, colour)
        x = np.where(C.mask[l][None], x, ghost_vals)
    m = C.mask[l]
    scale = _scale(Bfull[l][:, m], efull[l], coef, h)
    assert np.abs(got[:, m] - x[:, m]).max() <= 2e-13 * scale
