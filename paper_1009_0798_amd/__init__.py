"""MI355X library for the implicit ohmic-dissipation step of Matsumoto (PASJ
2011): one Crank-Nicolson step of dB/dt = -curl(eta curl B) on the 8^3-cell
blocks of a periodic AMR hierarchy, solved by multigrid on the GPU.

The Python layer only marshals arguments to the C ABI (include/ohm.h); fields
are torch tensors in GPU memory.  Functions keep the names of the C calls.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import CnOpts, CnStats, OhmError, OHM_F32, OHM_F64, check, dptr, host_doubles, lib, stream_ptr

BLOCK = 8
__all__ = ["Hierarchy", "ohm_fill_ghosts", "ohm_apply", "ohm_residual", "ohm_residual_noalloc", "ohm_smooth", "ohm_restrict",
           "ohm_prolong", "ohm_reflux", "ohm_cn_step", "ohm_explicit_step", "default_opts", "Workspace", "CnOpts",
           "OhmError", "to_blocks", "from_blocks"]


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return OHM_F64
    if t.dtype == torch.float32:
        return OHM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


class Hierarchy:
    """Handle over one or more periodic problems (``ohm_hier_create``).

    problems: list of (base_blocks (3 ints), dx0, [int32 [nb, 3] block coords per level]).
    """

    def __init__(self, problems, stream=None):
        L = lib()
        self.nprob = len(problems)
        descs = (_lib.ProblemDesc * self.nprob)()
        self._keep = []
        for d, (bb, dx0, levels) in zip(descs, problems):
            d.nlevels = len(levels)
            for a in range(3):
                d.base_blocks[a] = int(bb[a])
            d.dx0 = float(dx0)
            for l, blk in enumerate(levels):
                arr = np.ascontiguousarray(np.asarray(blk, dtype=np.int32).reshape(-1, 3))
                self._keep.append(arr)
                d.nblocks[l] = len(arr)
                d.block_ijk[l] = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        h = ctypes.c_void_p()
        check(L.ohm_hier_create(descs, self.nprob, stream_ptr(stream) if stream is not None else None,
                                ctypes.byref(h)))
        self.h = h
        self.nlevels = max(len(p[2]) for p in problems)
        self.min_level = 0
        self.prob_min_level = []
        for p in range(self.nprob):
            ml = ctypes.c_int32()
            check(L.ohm_hier_problem_info(h, p, 0, None, None, ctypes.byref(ml)))
            self.prob_min_level.append(ml.value)
            self.min_level = min(self.min_level, ml.value)

    def level_info(self, level):
        nb, nc, ng = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().ohm_hier_level_info(self.h, level, ctypes.byref(nb), ctypes.byref(nc), ctypes.byref(ng)))
        return nb.value, nc.value, ng.value

    def problem_info(self, prob, level):
        off, dims = ctypes.c_int64(), (ctypes.c_int32 * 3)()
        check(lib().ohm_hier_problem_info(self.h, prob, level, ctypes.byref(off), dims, None))
        return off.value, tuple(dims)

    def device_bytes(self):
        """Device bytes the handle itself holds (``ohm_hier_device_bytes``)."""
        n = ctypes.c_size_t()
        check(lib().ohm_hier_device_bytes(self.h, ctypes.byref(n)))
        return n.value

    def field(self, level, ncomp=3, dtype=None, fill=0.0):
        """A zero field of ``level`` in the library's layout."""
        import torch
        dtype = torch.float64 if dtype is None else dtype
        nb, nc, _ = self.level_info(level)
        shape = (ncomp, nb, BLOCK, BLOCK, BLOCK) if level >= 0 else (ncomp, nc)
        return torch.full(shape, fill, dtype=dtype, device="cuda")

    def ghost(self, level, ncomp=3, dtype=None):
        import torch
        dtype = torch.float64 if dtype is None else dtype
        _, _, ng = self.level_info(level)
        return torch.zeros((ncomp, max(ng, 1), BLOCK, BLOCK, BLOCK), dtype=dtype, device="cuda")

    def close(self):
        if getattr(self, "h", None):
            lib().ohm_hier_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _coef(h: Hierarchy, c):
    vals = np.broadcast_to(np.asarray(c, dtype=np.float64), (h.nprob,))
    return host_doubles(vals)


def ohm_fill_ghosts(h: Hierarchy, level, coarse, ghost, stream=None):
    ncomp = coarse.shape[0]
    check(lib().ohm_fill_ghosts(h.h, level, dptr(coarse), dptr(ghost), ncomp, _dtype_code(coarse), stream_ptr(stream)))


def ohm_apply(h: Hierarchy, level, B, eta, coef, out, B_ghost=None, eta_ghost=None, stream=None):
    check(lib().ohm_apply(h.h, level, dptr(B), dptr(B_ghost), dptr(eta), dptr(eta_ghost), _coef(h, coef), dptr(out),
                          _dtype_code(B), stream_ptr(stream)))


def ohm_residual(h: Hierarchy, level, B, S, eta, lam_dt, R=None, B_ghost=None, eta_ghost=None, norms=False,
                 stream=None):
    """Returns (nprob, 3, 2) numpy norms (sum R^2, max |R|) when norms=True."""
    nrm = (ctypes.c_double * (6 * h.nprob))() if norms else None
    check(lib().ohm_residual(h.h, level, dptr(B), dptr(B_ghost), dptr(S), dptr(eta), dptr(eta_ghost),
                             _coef(h, lam_dt), dptr(R), nrm, _dtype_code(B), stream_ptr(stream)))
    if norms:
        return np.array(nrm[:]).reshape(h.nprob, 3, 2)
    return None


def ohm_residual_noalloc(h: Hierarchy, level, B, S, eta, lam_dt, R=None, norms=None, B_ghost=None, eta_ghost=None,
                         stream=None):
    """``ohm_residual`` with its scratch in the library's static device array:
    ``norms`` (optional) is a float64 GPU tensor of nprob * 6 elements that
    receives (sum R^2, max |R|) per problem and component without a
    synchronisation."""
    if norms is not None:
        import torch
        if norms.dtype != torch.float64 or not norms.is_cuda or not norms.is_contiguous() or norms.numel() < 6 * h.nprob:
            raise ValueError(f"norms must be a contiguous float64 GPU tensor of at least {6 * h.nprob} elements")
    check(lib().ohm_residual_noalloc(h.h, level, dptr(B), dptr(B_ghost), dptr(S), dptr(eta), dptr(eta_ghost),
                                     _coef(h, lam_dt), dptr(R), dptr(norms), _dtype_code(B), stream_ptr(stream)))


def ohm_smooth(h: Hierarchy, level, B, S, eta, lam_dt, nsweeps, tmp, B_ghost=None, eta_ghost=None, stream=None,
               ordering=0):
    check(lib().ohm_smooth(h.h, level, dptr(B), dptr(B_ghost), dptr(S), dptr(eta), dptr(eta_ghost), _coef(h, lam_dt),
                           int(nsweeps), int(ordering), dptr(tmp), _dtype_code(B), stream_ptr(stream)))


def ohm_restrict(h: Hierarchy, fine_level, fine, coarse, stream=None):
    check(lib().ohm_restrict(h.h, fine_level, dptr(fine), dptr(coarse), fine.shape[0], _dtype_code(fine),
                             stream_ptr(stream)))


def ohm_prolong(h: Hierarchy, coarse_level, coarse, fine, accumulate=True, stream=None):
    check(lib().ohm_prolong(h.h, coarse_level, dptr(coarse), dptr(fine), coarse.shape[0], int(bool(accumulate)),
                            _dtype_code(coarse), stream_ptr(stream)))


def ohm_reflux(h: Hierarchy, level, B_coarse, eta_coarse, B_fine, eta_fine, coef, out, B_fine_ghost=None,
               eta_fine_ghost=None, zero_covered=True, stream=None):
    check(lib().ohm_reflux(h.h, level, dptr(B_coarse), dptr(eta_coarse), dptr(B_fine), dptr(B_fine_ghost),
                           dptr(eta_fine), dptr(eta_fine_ghost), _coef(h, coef), dptr(out), int(bool(zero_covered)),
                           _dtype_code(B_coarse), stream_ptr(stream)))


def default_opts(**kw) -> CnOpts:
    """The library's default ohm_cn_opts with the given fields replaced
    (``lam`` for lambda); an unknown name raises instead of being ignored."""
    o = CnOpts()
    lib().ohm_cn_default_opts(ctypes.byref(o))
    names = {f[0] for f in CnOpts._fields_}
    for k, v in kw.items():
        name = "lambda_" if k == "lam" else k
        if name not in names:
            raise TypeError(f"unknown Crank-Nicolson option {k!r}")
        setattr(o, name, v)
    return o


class Workspace:
    """Device workspace of ohm_cn_step, allocated through torch once per size."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.buf.data_ptr()
        off = (-base) % 256
        return base + off, self.buf.numel() - off


def _level_fields(h: Hierarchy, B, eta):
    """The step entry points read one B and one eta pointer per level of the
    handle: check the lists and tensors before their pointers are passed."""
    import torch
    if len(B) != h.nlevels or len(eta) != h.nlevels:
        raise ValueError(f"B and eta need one tensor per level ({h.nlevels}); got {len(B)} and {len(eta)}")
    for l, (b, e) in enumerate(zip(B, eta)):
        nb = h.level_info(l)[0]
        for name, t, n in (("B", b, 3 * nb * BLOCK ** 3), ("eta", e, nb * BLOCK ** 3)):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"{name}[{l}] must be a contiguous float64 GPU tensor of {n} elements; got "
                                 f"{t.dtype}, {t.device}, contiguous={t.is_contiguous()}, {t.numel()} elements")
    return ((ctypes.c_void_p * len(B))(*[b.data_ptr() for b in B]),
            (ctypes.c_void_p * len(eta))(*[e.data_ptr() for e in eta]))


def ohm_cn_step(h: Hierarchy, B, eta, dt, opts: CnOpts | None = None, workspace: Workspace | None = None,
                stream=None):
    """One CN step in place on the per-level FP64 fields ``B`` (list) with
    resistivity ``eta`` (list).  Returns (status, per-problem stats)."""
    L = lib()
    opts = default_opts() if opts is None else opts
    nb = ctypes.c_size_t()
    check(L.ohm_cn_workspace_size(h.h, ctypes.byref(opts), ctypes.byref(nb)))
    ws = workspace if workspace is not None else Workspace()
    Bp, Ep = _level_fields(h, B, eta)
    ptr, size = ws.get(nb.value)
    stats = (CnStats * h.nprob)()
    st = L.ohm_cn_step(h.h, Bp, Ep, _coef(h, dt), ctypes.byref(opts), ctypes.c_void_p(ptr), size, stats,
                       stream_ptr(stream))
    out = [dict(iters=s.iters, mg_apps=s.mg_apps, rel_res=s.rel_res, max_res=tuple(s.max_res)) for s in stats]
    if st not in (_lib.OHM_OK, _lib.OHM_ERR_NOCONV):
        check(st)
    return st, out


def ohm_explicit_step(h: Hierarchy, B, eta, dt, nsteps: int, workspace: Workspace | None = None, stream=None):
    """``nsteps`` explicit predictor-corrector steps of size ``dt`` in place on
    the per-level FP64 fields ``B`` (the comparison scheme of section 3.3)."""
    L = lib()
    nb = ctypes.c_size_t()
    check(L.ohm_explicit_workspace_size(h.h, ctypes.byref(nb)))
    ws = workspace if workspace is not None else Workspace()
    Bp, Ep = _level_fields(h, B, eta)
    ptr, size = ws.get(nb.value)
    check(L.ohm_explicit_step(h.h, Bp, Ep, _coef(h, dt), int(nsteps), ctypes.c_void_p(ptr), size,
                              stream_ptr(stream)))


def to_blocks(dense, block_ijk):
    """(ncomp, nz, ny, nx) tensor/array -> (ncomp, nb, 8, 8, 8) for the listed blocks."""
    ijk = np.asarray(block_ijk).reshape(-1, 3)
    parts = [dense[:, k * 8:(k + 1) * 8, j * 8:(j + 1) * 8, i * 8:(i + 1) * 8] for (i, j, k) in ijk]
    try:
        import torch
        if isinstance(dense, torch.Tensor):
            return torch.stack(parts, dim=1).contiguous()
    except ImportError:
        pass
    return np.ascontiguousarray(np.stack(parts, axis=1))


def from_blocks(blocks, block_ijk, dims):
    """Inverse of :func:`to_blocks` for a level that the blocks cover."""
    ijk = np.asarray(block_ijk).reshape(-1, 3)
    nx, ny, nz = dims
    try:
        import torch
        is_t = isinstance(blocks, torch.Tensor)
    except ImportError:
        is_t = False
    if is_t:
        out = torch.zeros((blocks.shape[0], nz, ny, nx), dtype=blocks.dtype, device=blocks.device)
    else:
        out = np.zeros((blocks.shape[0], nz, ny, nx), dtype=blocks.dtype)
    for n, (i, j, k) in enumerate(ijk):
        out[:, k * 8:(k + 1) * 8, j * 8:(j + 1) * 8, i * 8:(i + 1) * 8] = blocks[:, n]
    return out
