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


def cost_floor(orc, cl, poses):
    """Absolute rounding floor of the cost: each lambda_min is only defined to
    about eps * ||A_i|| by any backward-stable eigen-solver, so a cost that is
    zero in exact arithmetic is compared against 1e-14 * sum_i lambda_max(A_i)."""
    st = orc.voxel_stats(cl, poses)
    return 1e-14 * float(np.sum(st["lam"][:, 2]))


def resolved_prefix(tr, rep_ref, rtol=1e-11, floor=None):
    """Number of leading LM iterations whose accept / reject decision is
    resolved on both sides: the actual and the predicted cost changes exceed
    rtol of the cost.  Past that point the decision is set by rounding noise
    (several outcomes are correct) and traces are compared only at the end."""
    k = 0
    if floor is None:
        floor = 1e-12 * abs(rep_ref[0][0])
    for a, b in zip(tr, rep_ref):
        c = max(abs(b[0]), 1e-300)
        ok = True
        for r in (a, b):
            if r[6] != 0:      # failed factorization: decision is exact
                continue
            if abs(r[0] - r[1]) < rtol * c + floor or abs(r[7]) < rtol * c + floor:
                ok = False
        if not ok:
            break
        k += 1
    return k
