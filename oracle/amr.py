"""Oracle composite operator on a block-structured AMR hierarchy (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every level l is held as a dense periodic array over the whole box at its own
resolution h_l = dx0 / 2^l, together with
  mask[l]    -- cells that belong to a level-l block,
  covered[l] -- level-l cells that lie under a level-(l+1) block.
Leaf cells (mask & ~covered) are the unknowns of the composite system.

Composite operator (section 2.1 extended to the hierarchy):
 1. covered coarse B := mean of its 8 fine children (average down);
 2. every level-l cell outside the level's blocks (a ghost) gets the
    cell-centred trilinear interpolant of level l-1 -- for B and for eta.
    The paper does not state its coarse-fine interpolation; this reading is
    "parity unpinned" against the paper (pinned by invariants and by the
    paper's second-order convergence on its half-refined test, Fig. 5);
 3. face fluxes on each level by eqs. (4)-(6), (9)-(11);
 4. refluxing (section 4): on every coarse face next to a covered cell the
    coarse flux is the mean of the 4 fine fluxes on that face;
 5. divergence (8) at leaf cells.
"""
from __future__ import annotations

import numpy as np

from ohm_inputs import BLOCK, HierSpec

from . import ref
from . import mg


def face_restrict(Fd, d):
    """Mean of the 4 fine fluxes on each coarse face.  ``Fd`` is a fine flux
    array (3, NZ, NY, NX) through the faces p + e_d/2; the coarse face after
    coarse cell P along d is tiled by the fine faces after fine index 2 P_d + 1
    along d and 2 P_t, 2 P_t + 1 along the two other axes."""
    ax = 3 - d
    sl = [slice(None)] * 4
    sl[ax] = slice(1, None, 2)
    G = Fd[tuple(sl)]
    for a in (1, 2, 3):
        if a == ax:
            continue
        shp = list(G.shape)
        shp[a:a + 1] = [shp[a] // 2, 2]
        G = G.reshape(shp).mean(axis=a + 1)
    return G


class Composite:
    def __init__(self, spec: HierSpec):
        self.spec = spec
        self.L = spec.nlevels
        self.mask, self.covered = [], []
        for l in range(self.L):
            nx, ny, nz = spec.cells(l)
            m = np.zeros((nz, ny, nx), dtype=bool)
            for (i, j, k) in spec.levels[l]:
                m[k * BLOCK:(k + 1) * BLOCK, j * BLOCK:(j + 1) * BLOCK, i * BLOCK:(i + 1) * BLOCK] = True
            self.mask.append(m)
        for l in range(self.L):
            if l + 1 < self.L:
                fm = self.mask[l + 1]
                nz, ny, nx = self.mask[l].shape
                cov = fm.reshape(nz, 2, ny, 2, nx, 2).any(axis=(1, 3, 5))
                self.covered.append(cov)
            else:
                self.covered.append(np.zeros_like(self.mask[l]))
        self.leaf = [m & ~c for m, c in zip(self.mask, self.covered)]

    # -- conversions between block lists and dense level arrays -------------
    def to_dense(self, l, blocks, fill=np.nan):
        """blocks: [ncomp, nb, 8, 8, 8] or [nb, 8, 8, 8] -> dense level array."""
        scalar = blocks.ndim == 4
        b = blocks[None] if scalar else blocks
        nx, ny, nz = self.spec.cells(l)
        out = np.full((b.shape[0], nz, ny, nx), fill)
        for n, (i, j, k) in enumerate(self.spec.levels[l]):
            out[:, k * BLOCK:(k + 1) * BLOCK, j * BLOCK:(j + 1) * BLOCK,
                i * BLOCK:(i + 1) * BLOCK] = b[:, n]
        return out[0] if scalar else out

    def to_blocks(self, l, dense):
        scalar = dense.ndim == 3
        d = dense[None] if scalar else dense
        blk = self.spec.levels[l]
        out = np.empty((d.shape[0], len(blk), BLOCK, BLOCK, BLOCK))
        for n, (i, j, k) in enumerate(blk):
            out[:, n] = d[:, k * BLOCK:(k + 1) * BLOCK, j * BLOCK:(j + 1) * BLOCK,
                          i * BLOCK:(i + 1) * BLOCK]
        return out[0] if scalar else out

    # -- steps 1 and 2 --------------------------------------------------------
    def average_down(self, Bs):
        """Covered coarse cells := mean of the 8 children (finest first)."""
        Bs = [b.copy() for b in Bs]
        for l in range(self.L - 1, 0, -1):
            r = ref.restrict(np.where(self.mask[l], Bs[l], 0.0))
            cov = self.covered[l - 1]
            Bs[l - 1] = np.where(cov, r, Bs[l - 1])
        return Bs

    def ghost_values(self, coarse_complete):
        """Trilinear interpolant of a complete level-(l-1) array on level l."""
        return ref.prolong(coarse_complete)

    def fill_ghosts(self, Xs):
        """Return copies of the level arrays with every non-block cell replaced
        by the interpolant of the (already completed) next coarser level."""
        out = [Xs[0].copy()]
        for l in range(1, self.L):
            g = self.ghost_values(out[l - 1])
            out.append(np.where(self.mask[l], Xs[l], g))
        return out

    # -- steps 3-5 -------------------------------------------------------------
    def fluxes(self, Bs, etas, complete=False):
        if not complete:
            Bs = self.fill_ghosts(self.average_down(Bs))
            etas = self.fill_ghosts(etas)
        F = [ref.flux(Bs[l], etas[l], self.spec.dx(l)) for l in range(self.L)]
        for l in range(self.L - 1):
            cov = self.covered[l]
            for d in range(3):
                avg = face_restrict(F[l + 1][d], d)
                nbr = np.roll(cov, -1, axis=2 - d)    # is the cell across p + e_d/2 covered
                F[l][d] = np.where((cov | nbr)[None], avg, F[l][d])
        return F, Bs, etas

    def divF(self, Bs, etas):
        """(div F)_c at every cell of every level (meaningful at leaf cells)."""
        F, Bc, ec = self.fluxes(Bs, etas)
        return [ref.div(F[l], self.spec.dx(l)) for l in range(self.L)]

    def apply(self, Bs, etas, coef):
        """B + coef * div F on leaf cells; covered and ghost cells are 0."""
        D = self.divF(Bs, etas)
        return [np.where(self.leaf[l], Bs[l] + coef * D[l], 0.0) for l in range(self.L)]

    def source(self, bs, etas, dt, lam=0.5):
        return self.apply(bs, etas, -(1.0 - lam) * dt)

    def residual(self, Bs, Ss, etas, lam_dt):
        LB = self.apply(Bs, etas, lam_dt)
        return [np.where(self.leaf[l], Ss[l] - LB[l], 0.0) for l in range(self.L)]

    # -- leaf vectors ----------------------------------------------------------
    def pack(self, Xs):
        return np.concatenate([Xs[l][:, self.leaf[l]].ravel() for l in range(self.L)])

    def unpack(self, x, template=None):
        out, o = [], 0
        for l in range(self.L):
            n = int(self.leaf[l].sum())
            nx, ny, nz = self.spec.cells(l)
            a = np.zeros((3, nz, ny, nx)) if template is None else template[l].copy()
            a[:, self.leaf[l]] = x[o:o + 3 * n].reshape(3, n)
            out.append(a)
            o += 3 * n
        return out

    def volumes(self):
        """Cell volume of every packed unknown."""
        return np.concatenate([np.full(3 * int(self.leaf[l].sum()), self.spec.dx(l) ** 3)
                               for l in range(self.L)])

    def solve(self, Ss, etas, lam_dt, x0s=None, rtol=1e-13, maxit=2000):
        """Composite L^{-1} S by BiCGStab with a point-Jacobi preconditioner."""
        zero = [np.zeros_like(s) for s in Ss]
        Lop = lambda x: self.pack(self.apply(self.unpack(x, zero), etas, lam_dt))
        al = [ref.alpha(self.fill_ghosts(etas)[l], self.spec.dx(l), lam_dt) for l in range(self.L)]
        dinv = 1.0 / (1.0 + self.pack(al))
        M = lambda r: dinv * r
        x0 = self.pack(x0s) if x0s is not None else np.zeros(sum(3 * int(m.sum()) for m in self.leaf))
        x, hist = mg.bicgstab(Lop, self.pack(Ss), x0, M, rtol, maxit)
        return self.unpack(x, zero), hist

    def cn_step(self, bs, etas, dt, lam=0.5, rtol=1e-13):
        Ss = self.source(bs, etas, dt, lam)
        return self.solve(Ss, etas, lam * dt, x0s=bs, rtol=rtol)


class AMRMultigrid:
    """Multigrid for the composite correction equation L_comp e = r on an AMR
    hierarchy (section 2.2 and Table 1; the paper delegates the mechanics to
    its SFUMATO reference, which is not available, so the steps below are this
    project's reading, shared with the GPU solver).

    A composite V-cycle on levels 0..top, for the correction d of a current
    composite approximation z with residual t = r - L_comp z:
      down, m = top .. 1: nu sweeps on level m from d_m = 0 with zero
        coarse-fine ghosts; the level residual of d_m, restricted (mean of the
        8 children), becomes the right-hand side of the covered cells of level
        m - 1; the leaf cells of level m - 1 next to level m lose the change
        that d_m makes to the refluxed fluxes of their coarse-fine faces, taken
        with the same zero ghosts (the coarse correction is still zero);
      level 0: the base-grid multigrid (uniform periodic level, mg.fmg with
        n_base V-cycles of nu_base sweeps, or mg.vcycle) on the whole base grid;
      up, m = 1 .. top: d_m += trilinear prolongation of d_{m-1}; nu sweeps on
        level m with coarse-fine ghosts interpolated from d_{m-1}.
    FMG over the AMR levels (Table 1, first row): the right-hand side restricted
    to every level under finer blocks, the base grid solved alone, then for
    each finer level in turn the correction interpolated onto it and n_fmg
    composite V-cycles on the levels up to it; at the finest level n_mlat more
    composite V-cycles follow (second row).  Each composite V-cycle starts
    from the composite residual of the current approximation."""

    def __init__(self, comp: Composite, etas, lam_dt, nu=4, n_base=2, nu_base=2, base_fmg=True):
        self.C = comp
        self.etas = etas
        self.lam_dt = lam_dt
        self.L = comp.L
        self.nu = nu
        self.ef = comp.fill_ghosts(etas)
        self.base = mg.hierarchy(self.ef[0], comp.spec.dx(0), lam_dt)
        self.n_base, self.nu_base, self.base_fmg = n_base, nu_base, base_fmg
        # the composite operator of the levels 0..top, for every top
        self.sub = [Composite(HierSpec(comp.spec.base_blocks, comp.spec.dx0, comp.spec.levels[:top + 1]))
                    for top in range(self.L)]

    def smooth(self, m, d, t, ghost, n):
        """n red-black sweeps (eq. 19) on the cells of level m, ghosts fixed."""
        mask = self.C.mask[m][None]
        x = np.where(mask, d, ghost)
        for _ in range(n):
            for colour in (0, 1):
                x = ref.rb_halfsweep(x, t, self.ef[m], self.C.spec.dx(m), self.lam_dt, colour)
                x = np.where(mask, x, ghost)
        return np.where(mask, x, 0.0)

    def base_solve(self, t0):
        if self.base_fmg:
            return mg.fmg(self.base, t0, self.n_base, self.nu_base, self.nu_base)
        e = np.zeros_like(t0)
        for _ in range(self.n_base):
            e = e + mg.vcycle(self.base, t0 - self.base[0].L(e), self.nu_base, self.nu_base)
        return e

    def reflux_change(self, m, dm):
        """lam_dt times the divergence, at the leaf cells of level m - 1, of the
        refluxed coarse-fine face fluxes (mean of the 4 fine fluxes, eq. 11 and
        section 4) of a level-m correction dm taken with zero coarse-fine ghost
        values, the coarse correction being zero at that point of the cycle."""
        C = self.C
        Xs = [np.zeros((3,) + C.mask[l].shape) for l in range(self.L)]
        Xs[m] = np.where(C.mask[m][None], dm, 0.0)
        F, _, _ = C.fluxes(Xs, self.ef, complete=True)
        cov = C.covered[m - 1]
        Fm = []
        for dd in range(3):
            nbr = np.roll(cov, -1, axis=2 - dd)
            Fm.append(np.where((cov | nbr)[None], F[m - 1][dd], 0.0))
        D = ref.div(Fm, C.spec.dx(m - 1))
        return np.where(C.leaf[m - 1][None], self.lam_dt * D, 0.0)

    def vcycle(self, t, top):
        """Correction d on levels 0..top for the composite residual t."""
        C = self.C
        t = [x.copy() for x in t]
        d = [np.zeros_like(x) for x in t]
        for m in range(top, 0, -1):
            zero = np.zeros_like(d[m])
            d[m] = self.smooth(m, zero, t[m], zero, self.nu)
            res = t[m] - ref.apply(d[m], self.ef[m], C.spec.dx(m), self.lam_dt)
            rr = ref.restrict(np.where(C.mask[m][None], res, 0.0))
            t[m - 1] = np.where(C.covered[m - 1][None], rr, t[m - 1] - self.reflux_change(m, d[m]))
        d[0] = self.base_solve(t[0])
        for m in range(1, top + 1):
            g = ref.prolong(d[m - 1])
            d[m] = self.smooth(m, np.where(C.mask[m][None], d[m] + g, 0.0), t[m], g, self.nu)
        return d

    def residual(self, z, rf, top):
        """rf - L_comp z on the leaf cells of levels 0..top (level top has no
        finer level; its cells under finer blocks hold their own unknowns)."""
        S = self.sub[top]
        R = S.residual(z[:top + 1], rf[:top + 1], self.etas[:top + 1], self.lam_dt)
        return R + [np.zeros_like(x) for x in z[top + 1:]]

    def fmg(self, r, n_fmg=4, n_mlat=2):
        """e = L_comp^{-1} r by FMG over the AMR levels (see the class notes)."""
        C = self.C
        rf = [x.copy() for x in r]
        for m in range(self.L - 1, 0, -1):
            rr = ref.restrict(np.where(C.mask[m][None], rf[m], 0.0))
            rf[m - 1] = np.where(C.covered[m - 1][None], rr, rf[m - 1])
        z = [np.zeros_like(x) for x in r]
        z[0] = self.base_solve(rf[0])
        for top in range(1, self.L):
            z[top] = np.where(C.mask[top][None], ref.prolong(z[top - 1]), 0.0)
            for _ in range(n_fmg + (n_mlat if top == self.L - 1 else 0)):
                d = self.vcycle(self.residual(z, rf, top), top)
                z = [z[l] + d[l] if l <= top else z[l] for l in range(self.L)]
        return z

    def vcycles(self, r, n):
        """n composite V-cycles on all levels from a zero approximation."""
        z = [np.zeros_like(x) for x in r]
        for _ in range(n):
            d = self.vcycle(self.residual(z, r, self.L - 1), self.L - 1)
            z = [z[l] + d[l] for l in range(self.L)]
        return z
