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


def grad_abs_scale(orc, cl, poses):
    """G = || sum_i |g_i| ||_2: the summed absolute per-voxel gradient
    contributions (the oracle evaluated one voxel at a time).  Relative
    gradient errors are taken against G where the gradient itself cancels."""
    ends = np.flatnonzero(np.diff(cl.vox)) + 1
    starts = np.concatenate(([0], ends))
    stops = np.concatenate((ends, [cl.C]))
    acc = np.zeros(6 * cl.n_scans)
    for a, b in zip(starts, stops):
        sub = type(cl)(cl.vox[a:b].copy(), cl.scan[a:b].copy(), cl.n[a:b].copy(), cl.mu[a:b].copy(),
                       cl.S[a:b].copy(), cl.n_voxels, cl.n_scans)
        _, g, _, _ = orc.evaluate(orc.MM, sub, poses)
        acc += np.abs(g)
    return float(np.linalg.norm(acc))


def pose_diff(Pa, Pb):
    """(max rotation angle in rad, max translation difference) between pose sets."""
    Ra = np.asarray(Pa)[:, :9].reshape(-1, 3, 3)
    Rb = np.asarray(Pb)[:, :9].reshape(-1, 3, 3)
    c = (np.einsum("nij,nij->n", Ra, Rb) - 1.0) / 2.0
    ang = np.arccos(np.clip(c, -1.0, 1.0))
    dt = np.abs(np.asarray(Pa)[:, 9:] - np.asarray(Pb)[:, 9:]).max()
    return float(ang.max()), float(dt)


def align_to(Pa, Pb):
    """Pb moved by the one rigid motion G that maps its pose 0 onto Pa's pose 0
    (G = T_a0 T_b0^-1): removes the 6-dimensional gauge freedom of the cost
    before poses of two runs are compared."""
    Pa = np.asarray(Pa); Pb = np.asarray(Pb)
    Ra0 = Pa[0, :9].reshape(3, 3); ta0 = Pa[0, 9:]
    Rb0 = Pb[0, :9].reshape(3, 3); tb0 = Pb[0, 9:]
    Rg = Ra0 @ Rb0.T
    tg = ta0 - Rg @ tb0
    R = np.einsum("ij,njk->nik", Rg, Pb[:, :9].reshape(-1, 3, 3))
    t = Pb[:, 9:] @ Rg.T + tg
    return np.concatenate([R.reshape(-1, 9), t], axis=1)


def build_gpu_sums(ba, sc, dev, **kw):
    """Problem from a raw-sum scene (scenes.sums.SumsScene)."""
    import torch
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    if sc.n_windows > 1 and "scan_window" not in kw:
        kw = dict(kw, n_windows=sc.n_windows, scan_window=sc.scan_window)
    return ba.build_clusters_from_sums(t(sc.voxel, torch.int32), t(sc.scan, torch.int32),
                                       t(sc.count, torch.int64), t(sc.sum, torch.float64),
                                       t(sc.sumsq, torch.float64), sc.n_scans, sc.n_voxels, **kw)


def oracle_clusters_from_sums(orc, sc):
    """Oracle clusters of a raw-sum scene (the oracle centres the sums itself)."""
    order = np.lexsort((sc.scan, sc.voxel))
    mu, S = orc.center_raw_sums(sc.count[order], sc.sum[order], sc.sumsq[order])
    return orc.Clusters(sc.voxel[order].astype(np.int32), sc.scan[order].astype(np.int32),
                        sc.count[order].astype(np.int64), mu, S, sc.n_voxels, sc.n_scans)


def _worst_ratio(d, s):
    """max over blocks of d / s; a block whose scale is zero must be exact."""
    d = np.asarray(d, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    if np.any((s == 0) & (d != 0)):
        return float("inf")
    ok = s > 0
    return float(np.max(d[ok] / s[ok])) if np.any(ok) else 0.0


def block_err_g(g, g_ref, g_abs):
    """Largest per-pose gradient error, each pose's 6-vector against its own
    rounding scale: the norm of that pose's summed absolute per-cluster
    contributions (oracle.evaluate_abs).  Any summation order of the pose's
    terms is exact up to a multiple of eps times that scale, so a wrong block
    of a weakly observed pose cannot hide behind the strongly observed ones."""
    d = np.linalg.norm((np.asarray(g, dtype=np.float64).ravel() - np.asarray(g_ref).ravel()).reshape(-1, 6), axis=1)
    s = np.linalg.norm(np.asarray(g_abs).reshape(-1, 6), axis=1)
    return _worst_ratio(d, s)


def block_err_h(H, H_ref, H_abs):
    """Largest per-block Hessian error (Frobenius), each 6x6 block against the
    Frobenius norm of its summed absolute contributions.  MM: blocks [N][6][6];
    dense (6N, 6N): every (j, k) pose-pair block."""
    H = np.asarray(H, dtype=np.float64)
    H_ref = np.asarray(H_ref)
    H_abs = np.asarray(H_abs)
    if H_ref.ndim == 3:
        d = np.sqrt(((H.reshape(H_ref.shape) - H_ref) ** 2).sum(axis=(1, 2)))
        s = np.sqrt((H_abs ** 2).sum(axis=(1, 2)))
        return _worst_ratio(d, s)
    n = H_ref.shape[0] // 6
    blk = lambda A: A.reshape(n, 6, n, 6)
    d = np.sqrt(((blk(H) - blk(H_ref)) ** 2).sum(axis=(1, 3)))
    s = np.sqrt((blk(H_abs) ** 2).sum(axis=(1, 3)))
    return _worst_ratio(d, s)


def dense_backward_error(A, x, b):
    """Normwise backward error of a solve A x = b (Rigal-Gaches):
    ||A x - b||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    r = A @ x - b
    return float(np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()))


def lm_rounding_spread(orc, mode, cl, poses, iters, **kw):
    """Rounding sensitivity of the oracle's own LM run: the same run started
    from the poses moved by one ulp in every entry (up, then down).  Two
    correct FP64 executions of the iteration (different summation orders)
    differ by perturbations of this size, amplified by the same conditioning
    of the damped systems, so the spread is the yardstick for comparisons of
    whole LM runs where the steps amplify rounding beyond 1e-12.
    Returns (dtrace (iters, 8), dcost_final, dposes), the largest absolute
    differences of the perturbed runs from the unperturbed one."""
    P0 = np.asarray(poses, dtype=np.float64)
    P_a, rep_a, c_a = orc.lm(mode, cl, P0, iters, **kw)
    dtr = np.zeros((rep_a.shape[0], 8))
    dc = 0.0
    dP = np.zeros_like(P0)
    for direction in (np.inf, -np.inf):
        P_b, rep_b, c_b = orc.lm(mode, cl, np.nextafter(P0, direction), iters, **kw)
        k = min(rep_a.shape[0], rep_b.shape[0])
        dtr[:k] = np.maximum(dtr[:k], np.abs(rep_a[:k] - rep_b[:k]))
        dc = max(dc, abs(c_a - c_b))
        dP = np.maximum(dP, np.abs(P_a - P_b))
    return dtr, dc, dP
