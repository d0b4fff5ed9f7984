"""One red-black sweep (eq. 19) and the residual with its norms (eq. 20) on
full-size levels, checked at sampled cells against the oracle: the 128^3 and
256^3 levels on which the benchmark times the fused sweep (one launch per
sweep, 32-bit offsets), and the largest level class, an 832^3-cell level
(104^3 blocks, 576 M cells) whose FP64 field arrays exceed 4 GiB per
component, so the smoother leaves the fused sweep for one 64-bit-indexed
launch per colour.  At sampled cells: each sampled cell's neighbourhood of
radius 3 (a sweep reads radius 2) is copied into a 16^3 periodic box with the
colour parity kept, the oracle sweeps or evaluates the box, and its centre is
compared; the sample includes cells of the last blocks (at 832^3 more than
4 GiB, 2^32 bytes, into each component array).  The norms are checked as properties of
the returned residual (sum of squares and maximum per component)."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import ref

from gpu_util import announce

pytestmark = pytest.mark.gpu

RAD = 3


def _sample_cells(spec, rng, N):
    ijk = spec.levels[0]
    last = [tuple(int(v) for v in 8 * ijk[-1] + o) for o in ((0, 0, 0), (7, 7, 7), (3, 0, 7))]
    faces = [(8 * 9 - 1, 5, 9), (8 * 9, 5, 9), (0, 0, 0), (N - 1, N - 1, N - 1), (N - 1, 0, 7)]
    rand = [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(40)]
    return last + faces + rand


def _flat_index(lut, cells):
    """Element index of cells (M, 3) inside one component of the level array."""
    N = 8 * lut.shape[0]
    c = np.asarray(cells) % N
    b = lut[c[:, 2] >> 3, c[:, 1] >> 3, c[:, 0] >> 3].astype(np.int64)
    return b * 512 + (c[:, 2] & 7) * 64 + (c[:, 1] & 7) * 8 + (c[:, 0] & 7)


def _neighbourhoods(lut, cells):
    """(len(cells), 7^3) element indices of the radius-3 cube around each cell
    (periodic), ordered z, y, x."""
    d = np.arange(-RAD, RAD + 1)
    dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
    off = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)
    out = []
    for c in cells:
        out.append(_flat_index(lut, np.asarray(c) + off))
    return np.stack(out)


def _box(vals, centre_parity):
    """Embed a (ncomp, 7, 7, 7) neighbourhood in a 16^3 periodic box whose
    cell (x, y, z) has the colour parity of the global cell it stands for."""
    ncomp = vals.shape[0]
    box = np.zeros((ncomp, 16, 16, 16))
    x0 = 8 - RAD + centre_parity
    box[:, 8 - RAD:8 + RAD + 1, 8 - RAD:8 + RAD + 1, x0:x0 + 2 * RAD + 1] = vals
    return box, (8, 8, 8 + centre_parity)


@pytest.mark.parametrize("N", [128, 256, 832])
def test_sweep_and_residual_sampled_at_full_size(N):
    import torch
    import paper_1009_0798_amd as ohm
    NBA = N // 8
    announce(f"full size: {N}^3 level, {NBA ** 3} blocks, sampled sweep and residual")
    spec = gen.uniform_spec(N)
    assert (len(spec.levels[0]) * 512 * 8 > 2 ** 32) == (N == 832)
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    lut = np.empty((NBA, NBA, NBA), np.int32)
    ijk = spec.levels[0]
    lut[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = np.arange(len(ijk), dtype=np.int32)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    B = H.field(0, 3)
    B.normal_(generator=g)
    S = H.field(0, 3)
    S.normal_(generator=g)
    E = H.field(0, 1)
    E.uniform_(generator=g)
    E.mul_(-2.0 * np.log(10.0)).exp_()          # eta over two decades
    h = spec.dx0
    lam_dt = 0.5 * gen.explicit_dt(h, 1.0, 20.0)
    rng = np.random.default_rng(11)
    cells = _sample_cells(spec, rng, N)
    nbr = torch.from_numpy(_neighbourhoods(lut, cells)).cuda()
    Bf, Sf, Ef = B.view(3, -1), S.view(3, -1), E.view(1, -1)
    Bn = Bf[:, nbr].cpu().numpy()               # (3, M, 343)
    Sn = Sf[:, nbr].cpu().numpy()
    En = Ef[:, nbr].cpu().numpy()
    centre = torch.from_numpy(_flat_index(lut, cells)).cuda()
    if N == 832:
        assert int(centre.max()) * 8 > 2 ** 32

    announce(f"full size {N}^3: residual with norms")
    R = torch.empty_like(B)
    norms = ohm.ohm_residual(H, 0, B, S, E, lam_dt, R=R, norms=True)
    Rc = R.view(3, -1)[:, centre].cpu().numpy()
    for c in range(3):
        rc = R[c].double()
        assert abs(norms[0, c, 0] - float((rc * rc).sum())) <= 1e-11 * norms[0, c, 0]
        assert norms[0, c, 1] == float(rc.abs().max())
    del R

    announce(f"full size {N}^3: one red-black sweep")
    tmp = torch.empty_like(B)
    ohm.ohm_smooth(H, 0, B, S, E, lam_dt, 1, tmp)
    torch.cuda.synchronize()
    Bc = Bf[:, centre].cpu().numpy()
    del tmp

    announce(f"full size {N}^3: oracle on the sampled neighbourhoods")
    worst_r = worst_s = 0.0
    for m, cell in enumerate(cells):
        par = sum(cell) & 1
        b, ctr = _box(Bn[:, m].reshape(3, 7, 7, 7), par)
        s, _ = _box(Sn[:, m].reshape(3, 7, 7, 7), par)
        e, _ = _box(En[:, m].reshape(1, 7, 7, 7), par)
        e = e[0]
        e[e == 0] = 1.0                          # padding outside the neighbourhood
        z, y, x = ctr
        r_or = ref.residual(b, s, e, h, lam_dt)[:, z, y, x]
        b_or = ref.smooth(b, s, e, h, lam_dt, 1)[:, z, y, x]
        scale = np.abs(b).max() + np.abs(s).max()
        worst_r = max(worst_r, np.abs(Rc[:, m] - r_or).max() / scale)
        worst_s = max(worst_s, np.abs(Bc[:, m] - b_or).max() / scale)
        assert np.abs(Rc[:, m] - r_or).max() <= 1e-12 * scale, (cell, Rc[:, m], r_or)
        assert np.abs(Bc[:, m] - b_or).max() <= 1e-12 * scale, (cell, Bc[:, m], b_or)
    print("worst relative difference: residual", worst_r, "sweep", worst_s)
    H.close()
    del B, S, E, Bf, Sf, Ef, nbr, centre
    torch.cuda.empty_cache()
