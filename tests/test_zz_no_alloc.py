"""ohm_residual_noalloc (scratch in the library's static device array, device
norms, no synchronisation) against ohm_residual on the same inputs: the same
kernels in the same order, so R and the norms must agree bit for bit.  Two
calls in a row, the second on a smaller input, then an AMR level with ghost
blocks, a call captured into a HIP graph and replayed, then a level too large
for the array (rejected before any launch)."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import ref

from gpu_util import announce, cuda, dense_to_blocks

pytestmark = pytest.mark.gpu


def _problem(n, seed, D=3.0):
    spec = gen.uniform_spec(n)
    B = gen.divfree(n, 2.0, seed=seed)
    eta = gen.lognormal_eta(n, D, seed=seed + 1)
    dt = gen.explicit_dt(spec.dx0, 1.0, 50.0)
    S = ref.source(B, eta, spec.dx0, dt)
    return spec, B, eta, S, dt


def _compare(H, level, Bt, St, Et, lam_dt, Bg=None, Eg=None):
    import torch
    import paper_1009_0798_amd as ohm
    R1 = torch.empty_like(Bt)
    n1 = ohm.ohm_residual(H, level, Bt, St, Et, lam_dt, R=R1, B_ghost=Bg, eta_ghost=Eg, norms=True)
    R2 = torch.full_like(Bt, np.nan)
    n2 = torch.full((6 * H.nprob,), np.nan, dtype=torch.float64, device="cuda")
    ohm.ohm_residual_noalloc(H, level, Bt, St, Et, lam_dt, R=R2, norms=n2, B_ghost=Bg, eta_ghost=Eg)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2)
    got = n2.cpu().numpy().reshape(H.nprob, 3, 2)
    assert np.array_equal(got, n1), (got, n1)
    return R1, n1


def test_noalloc_residual_two_calls_then_smaller():
    import paper_1009_0798_amd as ohm
    announce("noalloc residual: 2 problems (32^3 + 24^3), then 16^3")
    specs, Bs, Es, Ss, dts = [], [], [], [], []
    for n, seed in ((32, 301), (24, 303)):
        spec, B, eta, S, dt = _problem(n, seed)
        specs.append(spec)
        Bs.append(dense_to_blocks(B, spec.levels[0]))
        Es.append(dense_to_blocks(eta, spec.levels[0])[None])
        Ss.append(dense_to_blocks(S, spec.levels[0]))
        dts.append(dt)
    H = ohm.Hierarchy([(s.base_blocks, s.dx0, s.levels) for s in specs])
    Bt, Et, St = cuda(np.concatenate(Bs, 1)), cuda(np.concatenate(Es, 1)), cuda(np.concatenate(Ss, 1))
    lam = [0.5 * d for d in dts]
    R, nrm = _compare(H, 0, Bt, St, Et, lam)
    # the norms are the sums and maxima of the returned residual
    Rh = R.cpu().numpy()
    o = 0
    for i, s in enumerate(specs):
        nb = len(s.levels[0])
        for c in range(3):
            r = Rh[c, o:o + nb]
            assert abs(nrm[i, c, 0] - np.sum(r * r)) <= 1e-12 * np.sum(r * r)
            assert nrm[i, c, 1] == np.abs(r).max()
        o += nb
    # second call, smaller input (the array still holds the first call's partials)
    spec, B, eta, S, dt = _problem(16, 305)
    H2 = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    _compare(H2, 0, cuda(dense_to_blocks(B, spec.levels[0])), cuda(dense_to_blocks(S, spec.levels[0])),
             cuda(dense_to_blocks(eta, spec.levels[0])[None]), 0.5 * dt)
    # FP32, norms only
    import torch
    Bt2 = cuda(dense_to_blocks(B, spec.levels[0])).float()
    St2 = cuda(dense_to_blocks(S, spec.levels[0])).float()
    Et2 = cuda(dense_to_blocks(eta, spec.levels[0])[None]).float()
    n1 = ohm.ohm_residual(H2, 0, Bt2, St2, Et2, 0.5 * dt, norms=True)
    n2 = torch.zeros(6, dtype=torch.float64, device="cuda")
    ohm.ohm_residual_noalloc(H2, 0, Bt2, St2, Et2, 0.5 * dt, norms=n2)
    assert np.array_equal(n2.cpu().numpy().reshape(1, 3, 2), n1)


def test_noalloc_residual_amr_level_with_ghosts():
    import paper_1009_0798_amd as ohm
    announce("noalloc residual: AMR level 1 with ghost blocks")
    spec = gen.config_amr2(n_base=16, extra_frac=0.2, seed=4)
    Bb, eb = gen.amr_fields(spec, p=2.0, seed=5)
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    Bc, Ec = cuda(Bb[0]), cuda(eb[0][None])
    B1, E1 = cuda(Bb[1]), cuda(eb[1][None])
    Bg, Eg = H.ghost(1, 3), H.ghost(1, 1)
    ohm.ohm_fill_ghosts(H, 1, Bc, Bg)
    ohm.ohm_fill_ghosts(H, 1, Ec, Eg)
    S1 = cuda(np.random.default_rng(9).standard_normal(tuple(B1.shape)))
    _compare(H, 1, B1, S1, E1, 1e-4, Bg, Eg)


def test_noalloc_residual_captured_in_a_graph():
    """18 problems (8^3 and 16^3, each its own lam_dt: the per-call scalars go
    to the device in two kernel-argument chunks), the call captured once into a
    HIP graph after an eager call, then replayed three times with new B written
    eagerly in between; every replay equals ohm_residual on the same inputs."""
    import torch
    import paper_1009_0798_amd as ohm
    announce("noalloc residual: 18 problems, captured into a graph, 3 replays")
    specs, Bs, Es, Ss, lam = [], [], [], [], []
    for i in range(18):
        n = 8 if i % 2 else 16
        spec, B, eta, S, dt = _problem(n, 400 + 2 * i)
        specs.append(spec)
        Bs.append(dense_to_blocks(B, spec.levels[0]))
        Es.append(dense_to_blocks(eta, spec.levels[0])[None])
        Ss.append(dense_to_blocks(S, spec.levels[0]))
        lam.append(0.5 * dt * (1.0 + 0.1 * i))
    H = ohm.Hierarchy([(s.base_blocks, s.dx0, s.levels) for s in specs])
    assert H.nprob == 18
    Bt, Et, St = cuda(np.concatenate(Bs, 1)), cuda(np.concatenate(Es, 1)), cuda(np.concatenate(Ss, 1))
    R = torch.empty_like(Bt)
    nrm = torch.zeros(6 * H.nprob, dtype=torch.float64, device="cuda")
    ohm.ohm_residual_noalloc(H, 0, Bt, St, Et, lam, R=R, norms=nrm)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ohm.ohm_residual_noalloc(H, 0, Bt, St, Et, lam, R=R, norms=nrm)
    rng = np.random.default_rng(17)
    for k in range(3):
        Bt.copy_(torch.from_numpy(rng.standard_normal(tuple(Bt.shape))).cuda())
        R.fill_(float("nan"))
        nrm.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        R1 = torch.empty_like(Bt)
        n1 = ohm.ohm_residual(H, 0, Bt, St, Et, lam, R=R1, norms=True)
        assert torch.equal(R, R1), k
        got = nrm.cpu().numpy().reshape(H.nprob, 3, 2)
        assert np.array_equal(got, n1), (k, got, n1)
    del g


def test_noalloc_residual_rejects_a_level_beyond_the_array():
    import torch
    import paper_1009_0798_amd as ohm
    from paper_1009_0798_amd import _lib
    announce("noalloc residual: oversize level rejected")
    nb = 45
    spec = gen.HierSpec((nb, nb, nb), 1.0 / (8 * nb), [gen.full_level((nb, nb, nb))])
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B = H.field(0, 3)
    E = H.field(0, 1, fill=1.0)
    norms = torch.zeros(6, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.OhmError) as err:
        ohm.ohm_residual_noalloc(H, 0, B, B, E, 1e-3, norms=norms)
    assert err.value.status == _lib.OHM_ERR_NOMEM
    # without norms the level needs only the coefficients: it runs
    R = torch.empty_like(B)
    ohm.ohm_residual_noalloc(H, 0, B, B, E, 1e-3, R=R)
    torch.cuda.synchronize()
    assert not R.any()
