"""Bottom-up multi-level voxelization and planarity selection (Sec. IV-A:
the L1 voxelization of Eq. 4, the level-up of Eq. 5, Alg. 1's
BottomUpVoxelization and Selection), written from the paper's definitions
with numpy in FP64.

TEST INFRASTRUCTURE ONLY: called by the test-suite and nothing else; the GPU
product path never imports it.

Definitions followed here (readings in the design notes):
  - world point of p in scan j: w = R_j p + t_j, each component evaluated as
    ((R_r0 p_x + R_r1 p_y) + R_r2 p_z) + t_r with every operation rounded
    (no fused multiply-add), so both implementations decide the same cells;
  - level-1 cell (Eq. 4): I^1 = floor(w / d) per axis;
  - level-k cell (Eq. 5): I^k = floor(I^(k-1) / 2);
  - a cluster is the (N, sum p, sum p p^T) of one scan's points in one cell,
    in the scan's body frame (Eq. 2); level-k clusters merge the level-(k-1)
    clusters of the same scan whose cells share a parent;
  - selection: the voxel covariance A of a cell's clusters mapped by the poses
    (Eq. 1, centred), eigenvalues l0 <= l1 <= l2; the cell is kept when
    l0 < tau * l1 (the paper's test), the cell holds at least three points
    and l1 > 1e-10 * l2 (readings: fewer than three points, or points on a
    line, span no plane, and such a covariance's l1 is only rounding), and (an
    option beyond the paper's rule) when at least min_scans scans observe it;
  - output: the kept cells of all levels concatenated in (level, cell, scan)
    order, voxel ids numbered densely in that order.
"""
from __future__ import annotations

import numpy as np

_SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
RANK2 = 1e-10   # l1 below this fraction of l2: rank below two, not a plane


def world_points(x, y, z, scan, poses):
    """w = R p + t per point, rounded after every operation."""
    P = np.asarray(poses, np.float64)[np.asarray(scan)]
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    w = np.empty((x.shape[0], 3))
    for r in range(3):
        w[:, r] = ((P[:, 3 * r] * x + P[:, 3 * r + 1] * y) + P[:, 3 * r + 2] * z) + P[:, 9 + r]
    return w


def _group(cell, scan):
    """Stable order by (cell x, cell y, cell z, scan) and the segment starts."""
    order = np.lexsort((scan, cell[:, 2], cell[:, 1], cell[:, 0]))
    c = cell[order]
    s = scan[order]
    head = np.ones(order.shape[0], bool)
    head[1:] = (c[1:] != c[:-1]).any(axis=1) | (s[1:] != s[:-1])
    starts = np.flatnonzero(head)
    return order, starts


def _level_clusters(cell, scan, count, s1, s2):
    """Merge rows with equal (cell, scan): counts and raw sums added."""
    order, starts = _group(cell, scan)
    return dict(cell=cell[order][starts], scan=scan[order][starts],
                count=np.add.reduceat(count[order], starts),
                sum=np.add.reduceat(s1[order], starts, axis=0),
                sumsq=np.add.reduceat(s2[order], starts, axis=0))


def select(cl, poses, tau, min_scans=1):
    """Per cell of a level: voxel covariance at the poses, its eigenvalues and
    the planarity decision.  Clusters must be in (cell, scan) order."""
    cell, scan, n = cl["cell"], cl["scan"], cl["count"].astype(np.float64)
    head = np.ones(cell.shape[0], bool)
    head[1:] = (cell[1:] != cell[:-1]).any(axis=1)
    vstart = np.flatnonzero(head)
    vid = np.cumsum(head) - 1
    mu = cl["sum"] / n[:, None]
    S = np.empty((n.shape[0], 3, 3))
    for q, (i, j) in enumerate(_SYM):
        S[:, i, j] = S[:, j, i] = cl["sumsq"][:, q] - n * mu[:, i] * mu[:, j]
    P = np.asarray(poses, np.float64)[scan]
    R = P[:, :9].reshape(-1, 3, 3)
    mw = np.einsum("kij,kj->ki", R, mu) + P[:, 9:]
    Sw = np.einsum("kia,kab,kjb->kij", R, S, R)
    V = vstart.shape[0]
    Nv = np.add.reduceat(n, vstart)
    mbar = np.add.reduceat(n[:, None] * mw, vstart, axis=0) / Nv[:, None]
    d = mw - mbar[vid]
    A = np.add.reduceat(Sw + n[:, None, None] * d[:, :, None] * d[:, None, :], vstart, axis=0) / Nv[:, None, None]
    lam = np.linalg.eigvalsh(A)
    n_scans = np.diff(np.append(vstart, cell.shape[0]))
    keep = ((Nv >= 3) & (lam[:, 1] > RANK2 * lam[:, 2]) & (lam[:, 0] < tau * lam[:, 1])
            & (n_scans >= min_scans))
    return dict(vstart=vstart, lam=lam, keep=keep, n_scans=n_scans, n_points=Nv.astype(np.int64), n_voxels=V)


def voxelize(x, y, z, scan, poses, d, levels, tau, min_scans=1):
    """Returns {"levels": [per level: clusters + selection], "out": concatenated kept clusters}."""
    scan = np.asarray(scan, np.int64)
    px, py, pz = (np.asarray(a, np.float64) for a in (x, y, z))
    w = world_points(px, py, pz, scan, poses)
    cell = np.floor(w / d).astype(np.int64)
    p = np.stack([px, py, pz], axis=1)
    s2 = np.stack([p[:, i] * p[:, j] for i, j in _SYM], axis=1)
    lv = []
    cl = _level_clusters(cell, scan, np.ones(p.shape[0], np.int64), p, s2)
    for k in range(1, levels + 1):
        if k > 1:
            prev = lv[-1]
            cl = _level_clusters(prev["cell"] >> 1, prev["scan"], prev["count"], prev["sum"], prev["sumsq"])
        cl.update(select(cl, poses, tau, min_scans))
        lv.append(cl)
    out = {k: [] for k in ("voxel", "scan", "count", "sum", "sumsq")}
    vlevel, vcell = [], []
    base = 0
    for k, cl in enumerate(lv):
        ends = np.append(cl["vstart"][1:], cl["cell"].shape[0])
        kept = np.flatnonzero(cl["keep"])
        for r, v in enumerate(kept):
            a, b = cl["vstart"][v], ends[v]
            out["voxel"].append(np.full(b - a, base + r, np.int64))
            out["scan"].append(cl["scan"][a:b])
            out["count"].append(cl["count"][a:b])
            out["sum"].append(cl["sum"][a:b])
            out["sumsq"].append(cl["sumsq"][a:b])
            vlevel.append(k + 1)
            vcell.append(cl["cell"][a])
        base += kept.shape[0]
    cat = lambda v, shape: np.concatenate(v) if v else np.zeros(shape)
    res = dict(voxel=cat(out["voxel"], (0,)).astype(np.int32), scan=cat(out["scan"], (0,)).astype(np.int32),
               count=cat(out["count"], (0,)).astype(np.int64), sum=cat(out["sum"], (0, 3)),
               sumsq=cat(out["sumsq"], (0, 6)), voxel_level=np.asarray(vlevel, np.int32),
               voxel_cell=np.asarray(vcell, np.int64).reshape(-1, 3), n_voxels=base)
    return dict(levels=lv, out=res)
