"""Oracle solvers on one uniform periodic level (FP64, plain numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The solution of one Crank-Nicolson step is the unique B with L B = S
(eqs. 12-14).  The oracle reaches it by any method; the multigrid pieces here
follow section 2.2-2.3 (averaging restriction, trilinear prolongation,
red-black smoother of eq. 19, iterative use of multigrid of eqs. 16-18) and the
readings listed in the design notes (coarsening depth, coarse resistivity,
coarsest solve).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ref


# --------------------------------------------------------------------------
# direct solve on small grids: the matrix of L, assembled by probing
# --------------------------------------------------------------------------
def _period(n: int) -> int:
    """Smallest divisor of n that is >= 3 (n itself for n < 3): cells of one
    probe colour are then at least 3 apart, so their +-1 stencils never share
    a row, even across the periodic seam."""
    for q in range(3, n + 1):
        if n % q == 0:
            return q
    return n


def assemble(eta, h, lam_dt) -> sp.csr_matrix:
    """Sparse matrix of L = I + lam_dt * div F (eq. 13), unknowns ordered as
    the flattened (3, nz, ny, nx) field.  Built by applying the oracle's L to
    coloured unit fields."""
    nz, ny, nx = eta.shape
    N = nx * ny * nz
    qx, qy, qz = _period(nx), _period(ny), _period(nz)
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    colour = (I % qx) + qx * ((J % qy) + qy * (K % qz))
    rows, cols, vals = [], [], []
    offs = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    for comp in range(3):
        for col in range(qx * qy * qz):
            sel = colour == col
            e = np.zeros((3, nz, ny, nx))
            e[comp][sel] = 1.0
            out = ref.apply(e, eta, h, lam_dt)
            ks, js, is_ = np.nonzero(sel)
            seen = set()
            for (a, b, c) in offs:
                key = ((a % nx) if nx < 3 else a, (b % ny) if ny < 3 else b, (c % nz) if nz < 3 else c)
                if key in seen:
                    continue
                seen.add(key)
                ri, rj, rk = (is_ + a) % nx, (js + b) % ny, (ks + c) % nz
                for rc in range(3):
                    v = out[rc, rk, rj, ri]
                    nzv = v != 0
                    rows.append(rc * N + (rk * ny + rj) * nx + ri)
                    cols.append(np.broadcast_to(comp * N + (ks * ny + js) * nx + is_, v.shape))
                    vals.append(np.where(nzv, v, 0.0))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = vals != 0
    M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(3 * N, 3 * N)).tocsr()
    M.sum_duplicates()
    return M


def direct_solve(eta, h, lam_dt, S):
    """L^{-1} S by a sparse LU factorisation (small grids only)."""
    M = assemble(eta, h, lam_dt).tocsc()
    return spla.spsolve(M, S.ravel()).reshape(S.shape)


# --------------------------------------------------------------------------
# multigrid on one periodic level
# --------------------------------------------------------------------------
def coarsen_ok(n) -> bool:
    """Reading of the unstated coarsening depth: halve while every axis is
    even, the coarse axes keep at least 2 cells, and the grid has more than
    64 cells."""
    nx, ny, nz = n
    return (nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0 and min(nx, ny, nz) >= 4
            and nx * ny * nz > 64)


class Level:
    def __init__(self, eta, h, lam_dt):
        self.eta, self.h, self.lam_dt = eta, h, lam_dt
        self.dense = None

    def L(self, x):
        return ref.apply(x, self.eta, self.h, self.lam_dt)

    def solve_exact(self, r):
        if self.dense is None:
            self.dense = np.linalg.inv(assemble(self.eta, self.h, self.lam_dt).toarray())
        return (self.dense @ r.ravel()).reshape(r.shape)


def hierarchy(eta, h, lam_dt):
    """Multigrid levels: rediscretised operator with the coarse resistivity the
    mean of the 8 children."""
    levels = [Level(eta, h, lam_dt)]
    while coarsen_ok(levels[-1].eta.shape[::-1]):
        lv = levels[-1]
        levels.append(Level(ref.restrict(lv.eta), 2 * lv.h, lam_dt))
    return levels


def vcycle(levels, r, nu1=2, nu2=2, l=0, ordering=0):
    """Correction-scheme V(nu1, nu2) cycle for L e = r starting from e = 0.
    The coarsest level is solved exactly (dense inverse).  ordering selects
    the smoother's colour classes (``ref.smooth``)."""
    lv = levels[l]
    if l == len(levels) - 1:
        return lv.solve_exact(r)
    e = np.zeros_like(r)
    e = ref.smooth(e, r, lv.eta, lv.h, lv.lam_dt, nu1, ordering)
    res = ref.residual(e, r, lv.eta, lv.h, lv.lam_dt)
    ec = vcycle(levels, ref.restrict(res), nu1, nu2, l + 1, ordering)
    e = ref.prolong(ec, e)
    e = ref.smooth(e, r, lv.eta, lv.h, lv.lam_dt, nu2, ordering)
    return e


def fmg(levels, r, n_v=1, nu1=2, nu2=2, ordering=0):
    """Full multigrid for L e = r: restrict r to every level, solve the
    coarsest, then on each finer level start from the prolonged coarse
    solution and run n_v V-cycles on the residual equation."""
    rs = [r]
    for l in range(1, len(levels)):
        rs.append(ref.restrict(rs[-1]))
    e = levels[-1].solve_exact(rs[-1])
    for l in range(len(levels) - 2, -1, -1):
        lv = levels[l]
        e = ref.prolong(e)
        for _ in range(n_v):
            res = ref.residual(e, rs[l], lv.eta, lv.h, lv.lam_dt)
            e = e + vcycle(levels, res, nu1, nu2, l, ordering)
    return e


# --------------------------------------------------------------------------
# outer iterations
# --------------------------------------------------------------------------
def _norm(x):
    return float(np.sqrt(np.sum(x * x)))


def iterative_mg(Lop, S, x, M, rtol=1e-13, maxit=200):
    """The paper's iterative use of multigrid, eqs. (16)-(18):
    R = S - L x;  x <- x + M(R);  repeat until |R|_2 <= rtol |S|_2."""
    nS = _norm(S)
    hist = []
    for it in range(maxit + 1):
        R = S - Lop(x)
        hist.append(_norm(R) / nS)
        if hist[-1] <= rtol or it == maxit:
            break
        x = x + M(R)
    return x, hist


def bicgstab(Lop, S, x, M, rtol=1e-13, maxit=200):
    """Right-preconditioned BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput.
    13, 1992) with the true residual checked at convergence."""
    nS = _norm(S)
    r = S - Lop(x)
    hist = [_norm(r) / nS]
    for _restart in range(5):
        rhat = r.copy()
        rho = alpha = omega = 1.0
        v = np.zeros_like(r)
        p = np.zeros_like(r)
        for _ in range(maxit):
            if hist[-1] <= rtol:
                break
            rho_new = float(np.sum(rhat * r))
            beta = (rho_new / rho) * (alpha / omega)
            rho = rho_new
            p = r + beta * (p - omega * v)
            ph = M(p)
            v = Lop(ph)
            alpha = rho / float(np.sum(rhat * v))
            s = r - alpha * v
            sh = M(s)
            t = Lop(sh)
            tt = float(np.sum(t * t))
            omega = float(np.sum(t * s)) / tt if tt > 0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            hist.append(_norm(r) / nS)
        r = S - Lop(x)
        hist.append(_norm(r) / nS)
        if hist[-1] <= rtol:
            break
    return x, hist


def cn_step(b, eta, h, dt, lam=0.5, rtol=1e-13, method="bicgstab", nu=2, maxit=200):
    """One step of eq. (7): solve L B = S with S from eq. (14), starting from
    B = b.  Returns (B, relative residual history)."""
    lam_dt = lam * dt
    S = ref.source(b, eta, h, dt, lam)
    levels = hierarchy(eta, h, lam_dt)
    Lop = levels[0].L
    M = lambda r: vcycle(levels, r, nu, nu)
    if method == "direct":
        return direct_solve(eta, h, lam_dt, S), []
    if method == "ir":
        return iterative_mg(Lop, S, b.copy(), M, rtol, maxit)
    return bicgstab(Lop, S, b.copy(), M, rtol, maxit)
