"""Helpers shared by the GPU tests: build a handle from a HierSpec and move
numpy fields between the dense level arrays of the oracle and the block layout
of the library (pure reshuffles, written here independently of both)."""
import sys

import numpy as np

B8 = 8


def dense_to_blocks(dense, ijk):
    d = dense[None] if dense.ndim == 3 else dense
    out = np.stack([d[:, k * B8:(k + 1) * B8, j * B8:(j + 1) * B8, i * B8:(i + 1) * B8] for (i, j, k) in ijk], axis=1)
    return np.ascontiguousarray(out[0] if dense.ndim == 3 else out)


def blocks_to_dense(blocks, ijk, dims, fill=np.nan):
    b = blocks[None] if blocks.ndim == 4 else blocks
    nx, ny, nz = dims
    out = np.full((b.shape[0], nz, ny, nx), fill)
    for n, (i, j, k) in enumerate(ijk):
        out[:, k * B8:(k + 1) * B8, j * B8:(j + 1) * B8, i * B8:(i + 1) * B8] = b[:, n]
    return out[0] if blocks.ndim == 4 else out


def dense_to_level(dense, h, level):
    """numpy dense (ncomp, nz, ny, nx) of problem 0 -> dense level layout (ncomp, ncells)."""
    d = dense[None] if dense.ndim == 3 else dense
    return d.reshape(d.shape[0], -1)


def hier(spec, stream=None):
    import paper_1009_0798_amd as ohm
    return ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)], stream)


def cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
