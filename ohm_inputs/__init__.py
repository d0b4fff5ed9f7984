"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random fields and block layouts.  It holds none of the
ohmic-dissipation arithmetic (no flux, no operator, no solver): both the HIP
library and the CPU oracle receive the arrays produced here as plain inputs.

Conventions
-----------
* A cell-centred field on a periodic box of ``n = (nx, ny, nz)`` cells is a
  float64 numpy array shaped ``(ncomp, nz, ny, nx)`` (x fastest).
* An AMR hierarchy is described by :class:`HierSpec`: level 0 tiles the box
  with 8^3-cell blocks; level ``l`` has cell width ``dx0 / 2**l`` and its blocks
  are listed by integer block coordinates in 8-cell units at that level.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BLOCK = 8


# --------------------------------------------------------------------------
# block layouts
# --------------------------------------------------------------------------
def _morton_key(ijk: np.ndarray) -> np.ndarray:
    """Interleave the bits of non-negative (i, j, k) triples (x lowest)."""
    key = np.zeros(len(ijk), dtype=np.int64)
    for bit in range(16):
        for d in range(3):
            key |= ((ijk[:, d].astype(np.int64) >> bit) & 1) << (3 * bit + d)
    return key


def morton_order(ijk: np.ndarray) -> np.ndarray:
    """Return ``ijk`` (int array [n, 3]) sorted along a Z-order curve."""
    ijk = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
    return ijk[np.argsort(_morton_key(ijk), kind="stable")]


def full_level(blocks_per_axis) -> np.ndarray:
    """All blocks of a box that is ``blocks_per_axis`` blocks wide, Morton order."""
    bx, by, bz = blocks_per_axis
    k, j, i = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    return morton_order(ijk)


@dataclasses.dataclass
class HierSpec:
    """Block structure of one periodic AMR problem (all cells cubic)."""

    base_blocks: tuple          # blocks per axis on level 0
    dx0: float                  # level-0 cell width
    levels: list                # list of int32 [nb, 3] block coordinates per level

    @property
    def nlevels(self) -> int:
        return len(self.levels)

    def cells(self, level: int) -> tuple:
        """Cells per axis of the whole box at ``level`` resolution (x, y, z)."""
        return tuple(BLOCK * b * (1 << level) for b in self.base_blocks)

    def dx(self, level: int) -> float:
        return self.dx0 / (1 << level)

    def leaf_cells(self) -> int:
        """Number of cells not covered by a finer level."""
        total = 0
        for l, blk in enumerate(self.levels):
            n = len(blk) * BLOCK ** 3
            if l + 1 < self.nlevels:
                n -= len(self.levels[l + 1]) * BLOCK ** 3 // 8
            total += n
        return total


def uniform_spec(n, dx=None) -> HierSpec:
    """Single-level hierarchy on an ``n`` (int or 3-tuple) cell periodic box."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    assert all(v % BLOCK == 0 for v in n), "box must be a whole number of 8^3 blocks"
    dx = 1.0 / n[0] if dx is None else dx
    bb = tuple(v // BLOCK for v in n)
    return HierSpec(bb, dx, [full_level(bb)])


def children_of(ijk: np.ndarray) -> np.ndarray:
    """The 8 finer blocks that exactly cover each block in ``ijk``."""
    ijk = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
    off = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int32)
    return (2 * ijk[:, None, :] + off[None, :, :]).reshape(-1, 3)


# --------------------------------------------------------------------------
# random fields
# --------------------------------------------------------------------------
def _wavenumbers(n):
    nx, ny, nz = n
    mx = np.fft.fftfreq(nx) * nx
    my = np.fft.fftfreq(ny) * ny
    mz = np.fft.fftfreq(nz) * nz
    MZ, MY, MX = np.meshgrid(mz, my, mx, indexing="ij")
    return MX, MY, MZ


def divfree_hat(n, p: float, seed: int) -> np.ndarray:
    """Fourier coefficients (complex [3, nz, ny, nx]) of :func:`divfree`."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, n[2], n[1], n[0]))
    W = np.fft.fftn(w, axes=(1, 2, 3))
    MX, MY, MZ = _wavenumbers(n)
    mag = np.sqrt(MX ** 2 + MY ** 2 + MZ ** 2)
    amp = np.zeros_like(mag)
    nz_ = mag > 0
    amp[nz_] = mag[nz_] ** (-p)
    W *= amp[None]
    # project out the part along the central-difference gradient direction so
    # that the sampled field has zero discrete (central) divergence
    c = np.stack([np.sin(2 * np.pi * MX / n[0]), np.sin(2 * np.pi * MY / n[1]),
                  np.sin(2 * np.pi * MZ / n[2])])
    c2 = (c ** 2).sum(0)
    ok = c2 > 1e-24
    dot = (c * W).sum(0)
    W = W - np.where(ok, c * dot / np.where(ok, c2, 1.0), 0.0)
    W[:, ~ok] = 0.0
    return W


def divfree(n, p: float = 2.0, seed: int = 0) -> np.ndarray:
    """Random periodic vector field with amplitude spectrum |m|^-p, zero mean,
    zero central-difference divergence, RMS 1.  Shape (3, nz, ny, nx)."""
    W = divfree_hat(n, p, seed)
    B = np.real(np.fft.ifftn(W, axes=(1, 2, 3)))
    rms = math.sqrt(float((B ** 2).mean()))
    return np.ascontiguousarray(B / rms if rms > 0 else B)


def divfree_sampled(n_base, p: float, seed: int, x, y, z):
    """Evaluate the band-limited :func:`divfree` field of an ``n_base`` box of
    unit-normalised coordinates at arbitrary points (x, y, z in cell units of
    the base grid, cell centres at integer + 1/2).  Used to sample one smooth
    field on several AMR levels."""
    n = (n_base, n_base, n_base) if np.isscalar(n_base) else tuple(n_base)
    W = divfree_hat(n, p, seed)
    B0 = np.real(np.fft.ifftn(W, axes=(1, 2, 3)))
    rms = math.sqrt(float((B0 ** 2).mean()))
    W = W / (rms * np.prod(n))
    MX, MY, MZ = _wavenumbers(n)
    # base cell centres sit at integer+1/2; the FFT sample j is at centre j+1/2
    keep = np.abs(W).max(axis=0) > 0
    mx, my, mz = MX[keep], MY[keep], MZ[keep]
    coef = W[:, keep]
    shape = np.broadcast(x, y, z).shape
    xs = (np.broadcast_to(x, shape) - 0.5).ravel()
    ys = (np.broadcast_to(y, shape) - 0.5).ravel()
    zs = (np.broadcast_to(z, shape) - 0.5).ravel()
    out = np.zeros((3, xs.size))
    chunk = 4096
    for s in range(0, xs.size, chunk):
        ph = np.exp(2j * np.pi * (np.outer(xs[s:s + chunk], mx / n[0])
                                  + np.outer(ys[s:s + chunk], my / n[1])
                                  + np.outer(zs[s:s + chunk], mz / n[2])))
        out[:, s:s + chunk] = np.real(ph @ coef.T).T
    return out.reshape((3,) + shape)


def lognormal_eta(n, decades: float, seed: int) -> np.ndarray:
    """Smooth random resistivity with max 1 spanning ``decades`` decades.
    Shape (nz, ny, nx)."""
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n[2], n[1], n[0]))
    MX, MY, MZ = _wavenumbers(n)
    filt = np.exp(-(MX ** 2 + MY ** 2 + MZ ** 2) / (2 * 4.0 ** 2))
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g = (g - g.min()) / max(g.max() - g.min(), 1e-300)
    return np.ascontiguousarray(10.0 ** (decades * (g - 1.0)))


def explicit_dt(h: float, eta_max: float, multiple: float) -> float:
    """``multiple`` times the explicit diffusion limit h^2 / (6 eta_max)."""
    return multiple * h * h / (6.0 * eta_max)


# --------------------------------------------------------------------------
# concrete workloads
# --------------------------------------------------------------------------
def uniform_problem(n, eta_decades=4.0, multiple=100.0, seed=0, p=2.0):
    """Generic uniform periodic workload: log-normal eta, k^-p div-free B."""
    spec = uniform_spec(n)
    h = spec.dx0
    eta = lognormal_eta(n, eta_decades, seed=2 * seed + 1) if eta_decades > 0 \
        else np.ones((n, n, n))
    B = divfree(n, p, seed=2 * seed + 2)
    return dict(spec=spec, B=B, eta=eta, dt=explicit_dt(h, float(eta.max()), multiple))


def config_fourier32():
    """32^3, eta = 1, three axis-aligned Fourier modes + 1e-3 div-free noise,
    dt = 20x the explicit limit, one CN step."""
    n = 32
    spec = uniform_spec(n)
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    B = np.zeros((3, n, n, n))
    B[1] += np.sin(2 * np.pi * X)
    B[2] += np.sin(4 * np.pi * Y) / 2
    B[0] += np.sin(6 * np.pi * Z) / 3
    B += 1e-3 * divfree(n, 0.0, seed=1)
    eta = np.ones((n, n, n))
    return dict(spec=spec, B=B, eta=eta, dt=explicit_dt(h, 1.0, 20.0), steps=1)


def config_lognormal128(n=128):
    """128^3, eta log-normal over 4 decades, div-free k^-2 B, dt = 100x the
    explicit limit, ten CN steps."""
    spec = uniform_spec(n)
    h = 1.0 / n
    eta = lognormal_eta(n, 4.0, seed=2)
    B = divfree(n, 2.0, seed=3)
    return dict(spec=spec, B=B, eta=eta, dt=explicit_dt(h, 1.0, 100.0), steps=10)


def dense_core_eta(x, y, z):
    """log10 eta = -3 + 2 (1 + tanh((0.2 - r) / 0.04)): 1e-3 outside, ~10 at r = 0."""
    r = np.sqrt(x * x + y * y + z * z)
    return 10.0 ** (-3.0 + 2.0 * (1.0 + np.tanh((0.2 - r) / 0.04)))


def level_centres(spec: HierSpec, level: int, origin=-0.5):
    """Physical cell-centre coordinates of every cell of a level's blocks.
    Returns (x, y, z), each [nb, 8, 8, 8] in (block, z, y, x) order."""
    blk = spec.levels[level]
    h = spec.dx(level)
    a = np.arange(BLOCK)
    gi = blk[:, 0, None, None, None] * BLOCK + a[None, None, None, :]
    gj = blk[:, 1, None, None, None] * BLOCK + a[None, None, :, None]
    gk = blk[:, 2, None, None, None] * BLOCK + a[None, :, None, None]
    x = origin + (gi + 0.5) * h
    y = origin + (gj + 0.5) * h
    z = origin + (gk + 0.5) * h
    return np.broadcast_arrays(x, y, z)


def config_amr2(n_base=64, extra_frac=0.2, seed=4):
    """Two-level hierarchy on [-1/2, 1/2)^3: base n_base^3, level 1 refines the
    central (n_base/16)^3 base blocks plus a seeded random ``extra_frac`` of the
    others; dense-core eta; dt = 20 x the explicit limit of the fine level at
    eta = 10."""
    bb = n_base // BLOCK
    lev0 = full_level((bb, bb, bb))
    c0 = bb // 2 - bb // 4
    core = [(i, j, k) for k in range(c0, c0 + bb // 2) for j in range(c0, c0 + bb // 2)
            for i in range(c0, c0 + bb // 2)]
    core_set = set(core)
    others = [tuple(b) for b in lev0 if tuple(b) not in core_set]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(others), size=int(round(extra_frac * len(others))), replace=False)
    refined = np.array(core + [others[i] for i in sorted(pick)], dtype=np.int32)
    lev1 = morton_order(children_of(refined))
    spec = HierSpec((bb, bb, bb), 1.0 / n_base, [lev0, lev1])
    return spec


def config_corner_gap():
    """Three levels on a 4^3-block base (32^3 cells on [-1/2, 1/2)^3): level 1
    is the 3^3 blocks (1..3)^3 without (3, 3, 3), level 2 the single block
    (4, 4, 4) over level-1 block (2, 2, 2).  Every face and edge neighbour of
    the level-2 block can be interpolated from level 1; its (+1, +1, +1)
    corner neighbour cannot (the cells it would need lie in the missing
    block)."""
    bb = (4, 4, 4)
    lev1 = np.array([(i, j, k) for k in range(1, 4) for j in range(1, 4) for i in range(1, 4)
                     if (i, j, k) != (3, 3, 3)], dtype=np.int32)
    lev2 = np.array([[4, 4, 4]], dtype=np.int32)
    return HierSpec(bb, 1.0 / 32, [full_level(bb), morton_order(lev1), lev2])


def amr_fields(spec: HierSpec, p=2.0, seed=5, eta_fn=dense_core_eta, origin=-0.5):
    """Sample one smooth div-free field (spectral, defined on the base grid) and
    eta at the cell centres of every level.  Covered coarse B = mean of its 8
    children.  Returns lists of [3, nb, 8, 8, 8] B and [nb, 8, 8, 8] eta."""
    n0 = spec.cells(0)
    Bs, etas = [], []
    for l in range(spec.nlevels):
        x, y, z = level_centres(spec, l, origin)
        # base-grid cell units: physical / dx0 - origin / dx0
        u = (x - origin) / spec.dx0
        v = (y - origin) / spec.dx0
        w = (z - origin) / spec.dx0
        Bs.append(divfree_sampled(n0, p, seed, u, v, w))
        etas.append(eta_fn(x, y, z))
    return Bs, etas


def refine_random(rng, parent_blocks: np.ndarray, parent_cells, frac: float,
                  margin: int = 1) -> np.ndarray:
    """Choose parent blocks to refine, covering about ``frac`` of the parent
    level's volume as one compact seeded patch, keeping a margin of ``margin``
    parent blocks inside the parent level (proper nesting).  Returns child
    block coordinates (Morton order)."""
    pset = {tuple(b) for b in parent_blocks}
    nbx, nby, nbz = (c // BLOCK for c in parent_cells)

    def interior(b):
        for dz in range(-margin, margin + 1):
            for dy in range(-margin, margin + 1):
                for dx in range(-margin, margin + 1):
                    q = ((b[0] + dx) % nbx, (b[1] + dy) % nby, (b[2] + dz) % nbz)
                    if q not in pset:
                        return False
        return True

    cand = [b for b in pset if interior(b)]
    if not cand:
        return np.zeros((0, 3), dtype=np.int32)
    target = max(1, int(round(frac * len(parent_blocks))))
    seed_b = cand[rng.integers(len(cand))]
    cand.sort(key=lambda b: sum(min(abs(b[d] - seed_b[d]), (nbx, nby, nbz)[d] - abs(b[d] - seed_b[d])) ** 2
                                for d in range(3)))
    chosen = np.array(cand[:target], dtype=np.int32)
    return morton_order(children_of(chosen))


def config_batched(nprob=256, seed=6, sizes=(16, 24, 32, 48, 64), decades=2.0, m_range=(10.0, 200.0)):
    """Independent uniform problems of uneven size: edge drawn uniformly from
    ``sizes``, log-normal eta over ``decades``, div-free k^-2 B, dt a
    log-uniform multiple in ``m_range`` of each problem's explicit limit."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nprob):
        n = int(rng.choice(sizes))
        m = float(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1]))))
        s1, s2 = int(rng.integers(1 << 30)), int(rng.integers(1 << 30))
        spec = uniform_spec(n)
        eta = lognormal_eta(n, decades, seed=s1)
        B = divfree(n, 2.0, seed=s2)
        out.append(dict(spec=spec, B=B, eta=eta, dt=explicit_dt(spec.dx0, float(eta.max()), m), m=m))
    return out


class FourierField:
    """A few random Fourier modes on the unit periodic box, evaluated at any
    points: B = sum_j a_j |k_j|^-p sin(2 pi k_j.x + phi_j) with polarisation a_j
    perpendicular to the integer wavevector k_j (continuously div-free), and a
    scalar g of the same kind for the resistivity."""

    def __init__(self, rng, nmodes=12, kmax=4, p=2.0):
        ks = []
        while len(ks) < nmodes:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(k != 0):
                ks.append(k)
        self.k = np.array(ks, dtype=float)
        kn = np.linalg.norm(self.k, axis=1)
        a = rng.standard_normal((nmodes, 3))
        a -= (a * self.k).sum(1, keepdims=True) * self.k / (kn ** 2)[:, None]
        self.a = a * (kn ** -p)[:, None]
        self.phi = rng.uniform(0, 2 * np.pi, nmodes)
        self.g = rng.standard_normal(nmodes) * kn ** -p

    def _phase(self, x, y, z):
        shape = np.broadcast(x, y, z).shape
        X = np.stack([np.broadcast_to(v, shape).ravel() for v in (x, y, z)], axis=1).astype(float)
        return 2 * np.pi * (X @ self.k.T) + self.phi, shape

    def vector(self, x, y, z):
        ph, shape = self._phase(x, y, z)
        return np.ascontiguousarray((np.sin(ph) @ self.a).T.reshape((3,) + shape))

    def scalar(self, x, y, z):
        ph, shape = self._phase(x, y, z)
        return (np.cos(ph) @ self.g).reshape(shape)


def amr_request(rng, n0, nlevels, decades, m, frac=0.125):
    """One serving request on the unit periodic box: n0^3 base cells (n0 a
    multiple of 8), ``nlevels`` levels, each finer level covering about
    ``frac`` of its parent level as one compact patch with a one-block nesting
    margin.  B and eta are smooth random Fourier fields sampled at every
    level's cell centres (covered coarse B = mean of its children); eta spans
    ``decades`` decades with max 1; dt = m x the explicit limit of the finest
    level.  Returns dict(spec, B (list of [3, nb, 8,8,8]), eta (list of
    [nb, 8,8,8]), dt)."""
    bb = (n0 // BLOCK,) * 3
    levels = [full_level(bb)]
    for l in range(1, nlevels):
        kids = refine_random(rng, levels[-1], tuple(BLOCK * b * (1 << (l - 1)) for b in bb), frac, margin=1)
        if len(kids) == 0:
            break
        levels.append(kids)
    spec = HierSpec(bb, 1.0 / n0, levels)
    F = FourierField(rng)
    Bs, gs = [], []
    for l in range(spec.nlevels):
        x, y, z = level_centres(spec, l, origin=0.0)
        Bs.append(F.vector(x, y, z))
        gs.append(F.scalar(x, y, z))
    lo = min(float(g.min()) for g in gs)
    hi = max(float(g.max()) for g in gs)
    es = [10.0 ** (decades * ((g - lo) / max(hi - lo, 1e-300) - 1.0)) for g in gs]
    # covered coarse cells hold the mean of their children
    for l in range(spec.nlevels - 1, 0, -1):
        par = {tuple(b): i for i, b in enumerate(spec.levels[l - 1])}
        for i, (bi, bj, bk) in enumerate(spec.levels[l]):
            pi_ = par[(bi >> 1, bj >> 1, bk >> 1)]
            ox, oy, oz = 4 * (bi & 1), 4 * (bj & 1), 4 * (bk & 1)
            f = Bs[l][:, i].reshape(3, 4, 2, 4, 2, 4, 2).mean(axis=(2, 4, 6))
            Bs[l - 1][:, pi_, oz:oz + 4, oy:oy + 4, ox:ox + 4] = f
    hf = spec.dx(spec.nlevels - 1)
    dt = explicit_dt(hf, 1.0, m)
    return dict(spec=spec, B=[np.ascontiguousarray(b) for b in Bs], eta=[np.ascontiguousarray(e) for e in es], dt=dt)


def amr_fields_fourier(spec: HierSpec, seed=5, eta_fn=dense_core_eta, origin=-0.5, nmodes=16):
    """Smooth div-free B (random Fourier modes on the unit box) and eta_fn at
    the cell centres of every level; covered coarse B = mean of its children.
    Returns per-level block arrays ([3, nb, 8, 8, 8], [nb, 8, 8, 8])."""
    F = FourierField(np.random.default_rng(seed), nmodes=nmodes)
    Bs, es = [], []
    for l in range(spec.nlevels):
        x, y, z = level_centres(spec, l, origin)
        Bs.append(F.vector(x - origin, y - origin, z - origin))
        es.append(np.ascontiguousarray(eta_fn(x, y, z)))
    for l in range(spec.nlevels - 1, 0, -1):
        par = {tuple(b): i for i, b in enumerate(spec.levels[l - 1])}
        for i, (bi, bj, bk) in enumerate(spec.levels[l]):
            pi_ = par[(bi >> 1, bj >> 1, bk >> 1)]
            ox, oy, oz = 4 * (bi & 1), 4 * (bj & 1), 4 * (bk & 1)
            Bs[l - 1][:, pi_, oz:oz + 4, oy:oy + 4, ox:ox + 4] = Bs[l][:, i].reshape(3, 4, 2, 4, 2, 4, 2).mean(axis=(2, 4, 6))
    return [np.ascontiguousarray(b) for b in Bs], es


def config_e8(n=64, L=8.0):
    """The explicit-comparison test of section 3.3: periodic box [-L/2, L/2)^3
    resolved by n^3 cells, eta = exp(-r^2), B = (0, 0, exp(-(x^2 + y^2))),
    run to t = 1 with dt = 1e-3 (explicit) and 1e-1 (implicit)."""
    h = L / n
    c = -L / 2 + (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    eta = np.exp(-(X * X + Y * Y + Z * Z))
    B = np.zeros((3, n, n, n))
    B[2] = np.exp(-(X * X + Y * Y))
    return dict(spec=uniform_spec(n, dx=h), B=B, eta=eta, t_end=1.0, dt_explicit=1e-3, dt_implicit=1e-1)
