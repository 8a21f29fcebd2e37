"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np


def to_dev(sc, dev):
    import torch
    f = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    return (f(sc.x, torch.float64), f(sc.y, torch.float64), f(sc.z, torch.float64), f(sc.scan, torch.int32),
            f(sc.voxel, torch.int32))


def build_gpu(ba, sc, dev, **kw):
    x, y, z, s, v = to_dev(sc, dev)
    return ba.build_clusters(x, y, z, s, v, sc.n_scans, sc.n_voxels, **kw)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def grad_rel_err(g, g_ref, g_abs_scale):
    """Relative gradient error: against ||g_ref|| when that is not tiny compared
    with the summed absolute contributions, else against that scale."""
    d = np.linalg.norm(np.asarray(g) - np.asarray(g_ref))
    nref = np.linalg.norm(g_ref)
    return d / max(nref, 1e-3 * g_abs_scale, 1e-300)
