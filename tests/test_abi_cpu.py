"""C-ABI contract checks that need no GPU: the library loads, exports every
call of include/ohm.h, and rejects bad hierarchies on the host before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import ohm_inputs as gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_calls():
    src = open(os.path.join(ROOT, "include", "ohm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ohm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_seven_calls():
    calls = _header_calls()
    for name in ["ohm_apply", "ohm_residual", "ohm_smooth", "ohm_restrict", "ohm_prolong", "ohm_fill_ghosts",
                 "ohm_cn_step"]:
        assert name in calls


def test_library_exports_every_declared_symbol():
    from paper_1009_0798_amd import _lib
    L = _lib.lib()
    for name in _header_calls():
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == sorted(_header_calls())


def _create(problems):
    from paper_1009_0798_amd import _lib
    L = _lib.lib()
    descs = (_lib.ProblemDesc * len(problems))()
    keep = []
    for d, (bb, dx0, levels) in zip(descs, problems):
        d.nlevels = len(levels)
        for a in range(3):
            d.base_blocks[a] = bb[a]
        d.dx0 = dx0
        for l, blk in enumerate(levels):
            arr = np.ascontiguousarray(np.asarray(blk, dtype=np.int32).reshape(-1, 3))
            keep.append(arr)
            d.nblocks[l] = len(arr)
            d.block_ijk[l] = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    st = L.ohm_hier_create(descs, len(problems), None, ctypes.byref(h))
    return st, L.ohm_last_error().decode()


def test_rejects_incomplete_base_level():
    lev0 = gen.full_level((2, 2, 2))[:-1]
    st, msg = _create([((2, 2, 2), 0.1, [lev0])])
    assert st == 2 and "level 0" in msg


def test_rejects_duplicate_and_outside_blocks():
    lev0 = gen.full_level((2, 2, 1))
    dup = np.concatenate([lev0[:-1], lev0[:1]])
    st, msg = _create([((2, 2, 1), 0.1, [dup])])
    assert st == 2 and "duplicate" in msg
    bad = lev0.copy()
    bad[0] = (5, 0, 0)
    st, msg = _create([((2, 2, 1), 0.1, [bad])])
    assert st == 2 and "outside" in msg


def test_rejects_improper_nesting():
    """A level-2 block at the edge of level 1 has coarse-fine ghosts whose
    interpolation would need level-1 cells that do not exist."""
    lev0 = gen.full_level((4, 4, 4))
    lev1 = gen.children_of(np.array([[1, 1, 1]], dtype=np.int32))   # 8 blocks over base block (1,1,1)
    lev2 = gen.children_of(np.array([[2, 2, 2]], dtype=np.int32))   # at the corner of level 1
    st, msg = _create([((4, 4, 4), 0.1, [lev0, lev1, lev2])])
    assert st == 2 and "nested" in msg


def test_rejects_bad_arguments():
    st, msg = _create([((0, 1, 1), 0.1, [gen.full_level((1, 1, 1))])])
    assert st == 1
    st, msg = _create([((1, 1, 1), -1.0, [gen.full_level((1, 1, 1))])])
    assert st == 1 and "dx0" in msg


def test_null_handle_errors():
    from paper_1009_0798_amd import _lib
    L = _lib.lib()
    assert L.ohm_hier_level_info(None, 0, None, None, None) == 1
    assert "NULL" in L.ohm_last_error().decode()
    o = _lib.CnOpts()
    L.ohm_cn_default_opts(ctypes.byref(o))
    assert o.lambda_ == 0.5 and o.rtol == 1e-10


def test_default_opts_fields_and_unknown_names():
    """The binding's option structure matches the library's defaults field by
    field (a shifted field would show here), and a misspelled option raises."""
    import paper_1009_0798_amd as ohm
    o = ohm.default_opts()
    assert (o.lambda_, o.rtol, o.max_iters, o.nu_pre, o.nu_post, o.n_vcycles, o.cycle, o.outer, o.precision,
            o.coarse_sweeps, o.nu_coarse, o.graph, o.ordering) == (0.5, 1e-10, 100, 2, 2, 1, 0, 1, 0, 16, 0, 1, 0)
    assert ohm.default_opts(lam=1.0, ordering=1).ordering == 1
    with pytest.raises(TypeError, match="nu_pree"):
        ohm.default_opts(nu_pree=3)


def _slab_levels(depth, shift_last=0):
    """64 x 1 x 1 base blocks; level l refines a 4-block-wide slab in x over all
    of y and z, nested in level l-1 with a one-coarse-block margin (so every
    level but the last is properly nested; shift_last = 1 moves the last one
    to the edge of its parent slab)."""
    bb = (64, 1, 1)
    levels = [gen.full_level(bb)]
    a = 10
    for l in range(1, depth + 1):
        a = 2 * a + 2 if l > 1 else a
        x0 = a - (shift_last if l == depth else 0)
        n = 1 << l
        levels.append(np.array([(x, y, z) for z in range(n) for y in range(n) for x in range(x0, x0 + 4)],
                               dtype=np.int32))
        a = x0
    return bb, levels


def test_deep_levels_use_the_sparse_block_index():
    """Level 7 of a 64 x 1 x 1-block base spans 8192 x 128 x 128 block
    positions, more than the dense block index of the handle build holds
    (2^24), so its lookups go through the hash map: a properly built chain is
    accepted up to validation, a duplicate block there and a block whose
    coarser cover is missing are still rejected."""
    bb, levels = _slab_levels(7)
    dup = levels[:-1] + [np.concatenate([levels[-1], levels[-1][5:6]])]
    st, msg = _create([(bb, 1.0, dup)])
    assert st == 2 and "duplicate" in msg and "level 7" in msg, msg
    bb, bad = _slab_levels(7, shift_last=1)
    st, msg = _create([(bb, 1.0, bad)])
    assert st == 2 and "level 7" in msg and "not properly nested" in msg, msg


def test_step_bindings_check_the_level_lists():
    """The step entry points take one B and one eta pointer per level of the
    handle; the binding refuses a list of the wrong length (the library would
    read past it) and a tensor of the wrong type, place or size, before any
    pointer is passed.  A stand-in handle (two levels of 5 and 3 blocks)
    serves, so no device is needed."""
    import torch
    import paper_1009_0798_amd as ohm

    class Handle:
        nlevels = 2

        def level_info(self, l):
            return (5, 5 * 512, 0) if l == 0 else (3, 3 * 512, 0)

    h = Handle()
    B = [torch.zeros(3, 5, 8, 8, 8, dtype=torch.float64), torch.zeros(3, 3, 8, 8, 8, dtype=torch.float64)]
    E = [torch.ones(1, 5, 8, 8, 8, dtype=torch.float64), torch.ones(1, 3, 8, 8, 8, dtype=torch.float64)]
    with pytest.raises(ValueError, match="one tensor per level"):
        ohm._level_fields(h, B[:1], E)
    with pytest.raises(ValueError, match="one tensor per level"):
        ohm._level_fields(h, B, E + E[:1])
    # host tensors are refused (the library takes device pointers)
    with pytest.raises(ValueError, match=r"B\[0\] must be a contiguous float64 GPU tensor of 7680"):
        ohm._level_fields(h, B, E)
