"""Seeded synthetic scenes generated directly as raw-sum point clusters.

The largest workloads (a 2000-pose city-scale map with 1M planes, a batch of
256 windows, served request streams) hold 0.3-2 billion virtual points, too
many to materialise.  This module draws every (voxel, scan) cluster's
statistics exactly instead of its points: the in-plane coordinates of the
virtual points follow a Gaussian with the variance of the uniform 1 m patch
(patch^2 / 12 per axis) and the normal offset N(0, sigma^2), so the sample
mean of n points is normal with covariance D / n and the centred scatter
matrix is Wishart(D, n - 1), independent of the mean; the scatter is drawn
with the Bartlett decomposition (Bartlett 1933; Smith & Hocking 1972).  The
cluster is then handed over in the paper's raw-sum form (N, sum p, sum p p^T)
in the scan's body frame, p = R^T (x - t).

Like the point generator, this module only synthesises inputs; it performs
none of the method's arithmetic.  All randomness comes from numpy's
Philox4x32-10 counter-based generator keyed by the seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

from . import _pack, _perturb, _rng, _rz, _unit_normals, _inplane_basis


@dataclass
class SumsScene:
    name: str
    seed: int
    voxel: np.ndarray        # (C,) int32
    scan: np.ndarray         # (C,) int32
    count: np.ndarray        # (C,) int64, N_ij >= 4
    sum: np.ndarray          # (C, 3) float64: sum p (body frame)
    sumsq: np.ndarray        # (C, 6) float64: sum p p^T [xx xy xz yy yz zz]
    n_scans: int
    n_voxels: int
    poses_true: np.ndarray   # (n_scans, 12)
    poses_init: np.ndarray   # (n_scans, 12)
    n_windows: int = 1
    scan_window: np.ndarray | None = None   # (n_scans,) int32, non-decreasing
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self) -> int:
        return int(self.voxel.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.count.sum())


def _cluster_sums(rng, centres, normals, obs_v, obs_s, npts, r_true, t_true, sigma, patch=1.0,
                  chunk=1 << 20):
    """Raw sums of every observation (obs_v[k], obs_s[k]) with npts[k] virtual points."""
    e1, e2 = _inplane_basis(normals)
    sd = (patch / math.sqrt(12.0), patch / math.sqrt(12.0), sigma)
    C = obs_v.shape[0]
    s1 = np.empty((C, 3))
    s2 = np.empty((C, 6))
    for a in range(0, C, chunk):
        b = min(C, a + chunk)
        v, s, n = obs_v[a:b], obs_s[a:b], npts[a:b].astype(np.float64)
        k = b - a
        R = r_true[s]                                   # (k, 3, 3), body -> world
        cols = (e1[v], e2[v], normals[v])               # world plane frame
        # Bb[:, i, l] = (R^T col_l)_i * sd_l : plane axes in the body frame, scaled by D^(1/2)
        Bb = np.empty((k, 3, 3))
        for l in range(3):
            c = cols[l]
            for i in range(3):
                Bb[:, i, l] = sd[l] * (R[:, 0, i] * c[:, 0] + R[:, 1, i] * c[:, 1] + R[:, 2, i] * c[:, 2])
        dc = centres[v] - t_true[s]
        z = rng.standard_normal((k, 3)) / np.sqrt(n)[:, None]
        mu = np.empty((k, 3))
        for i in range(3):
            mu[:, i] = (Bb[:, i, 0] * z[:, 0] + Bb[:, i, 1] * z[:, 1] + Bb[:, i, 2] * z[:, 2]
                        + R[:, 0, i] * dc[:, 0] + R[:, 1, i] * dc[:, 1] + R[:, 2, i] * dc[:, 2])
        # Bartlett factor L (lower triangular) of a Wishart(I, n - 1) draw
        dof = n - 1.0
        l00 = np.sqrt(rng.chisquare(dof))
        l11 = np.sqrt(rng.chisquare(dof - 1.0))
        l22 = np.sqrt(rng.chisquare(dof - 2.0))
        l10, l20, l21 = rng.standard_normal((3, k))
        # F = Bb L ; centred scatter S = F F^T
        F = np.empty((k, 3, 3))
        for i in range(3):
            F[:, i, 0] = Bb[:, i, 0] * l00 + Bb[:, i, 1] * l10 + Bb[:, i, 2] * l20
            F[:, i, 1] = Bb[:, i, 1] * l11 + Bb[:, i, 2] * l21
            F[:, i, 2] = Bb[:, i, 2] * l22
        s1[a:b] = n[:, None] * mu
        for q, (i, j) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
            Sij = F[:, i, 0] * F[:, j, 0] + F[:, i, 1] * F[:, j, 1] + F[:, i, 2] * F[:, j, 2]
            s2[a:b, q] = Sij + n * mu[:, i] * mu[:, j]
    return s1, s2


def _pool(workers: int):
    """Worker processes for the scene generators.  They are started fresh
    (spawn), never forked: the caller may already hold a GPU context, which a
    forked child must not inherit."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    return ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))


def _truncated_geometric(rng, p, m_max, size):
    k = np.arange(1, m_max + 1)
    pk = (1 - p) ** (k - 1) * p
    pk /= pk.sum()
    return rng.choice(k, size=size, p=pk)


def _nearest_observers(t_true, centres, m, obs_radius):
    """The m nearest poses within obs_radius of each plane (at least the nearest one)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(t_true)
    n_planes = centres.shape[0]
    kq = int(min(m.max(), t_true.shape[0]))
    import os
    dist, idx = tree.query(centres, k=kq, distance_upper_bound=obs_radius, workers=min(16, os.cpu_count() or 1))
    dist = dist.reshape(n_planes, kq)
    idx = idx.reshape(n_planes, kq)
    valid = np.isfinite(dist) & (np.arange(kq)[None, :] < m[:, None])
    none = ~valid.any(axis=1)
    if none.any():
        _, nn = tree.query(centres[none], k=1)
        idx[none, 0] = nn
        valid[none, 0] = True
    big = np.iinfo(np.int64).max
    sidx = np.where(valid, idx, big)
    sidx.sort(axis=1)
    keep = sidx != big
    obs_s = sidx[keep].astype(np.int32)
    obs_v = np.repeat(np.arange(n_planes, dtype=np.int32), keep.sum(axis=1))
    return obs_v, obs_s


def _loglog_counts(rng, lo, hi, size):
    n = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)
    return np.clip(n, lo, hi)


def _city_trajectory(n_poses, width=5000.0, height=1000.0):
    """A closed width x height rectangular loop with a cross street through its
    middle, origin at a corner; poses evenly spaced along the route."""
    segs = [((0, 0), (width, 0)), ((width, 0), (width, height)), ((width, height), (0, height)),
            ((0, height), (0, 0)), ((width / 2, 0), (width / 2, height))]
    lens = [math.hypot(b[0] - a[0], b[1] - a[1]) for a, b in segs]
    total = sum(lens)
    s = np.arange(n_poses) * (total / n_poses)
    pts = np.zeros((n_poses, 3))
    head = np.zeros(n_poses)
    acc = np.cumsum([0.0] + lens)
    for k, sk in enumerate(s):
        i = int(np.searchsorted(acc, sk, side="right") - 1)
        i = min(i, len(segs) - 1)
        (ax, ay), (bx, by) = segs[i]
        f = (sk - acc[i]) / lens[i]
        pts[k, 0] = ax + f * (bx - ax)
        pts[k, 1] = ay + f * (by - ay)
        head[k] = math.atan2(by - ay, bx - ax)
    return pts, head


def city_config(seed: int = 3000, n_scans: int = 2000, n_planes: int = 1_000_000, geom_p: float = 0.15,
                m_max: int = 30, pts_range=(20, 1000), sigma: float = 0.03, rot_bound_deg: float = 1.0,
                trans_bound: float = 0.10, place_radius: float = 40.0, obs_radius: float = 80.0,
                name: str | None = None) -> SumsScene:
    """City-scale precision-form workload: ``n_scans`` poses on a 5 km x 1 km
    loop with a cross street (coordinates spanning 5 km from the origin),
    ``n_planes`` planes each centred within ``place_radius`` of a random
    anchor pose and observed by its m nearest poses within ``obs_radius``
    (m ~ geometric(p) truncated to [1, m_max]), N_ij log-uniform in
    ``pts_range``, N(0, sigma) normal noise, +-1 deg / +-10 cm perturbation."""
    rng = _rng(seed)
    t_true, head = _city_trajectory(n_scans)
    r_true = _rz(head)
    nrm = _unit_normals(rng, n_planes)
    anchor = rng.integers(0, n_scans, size=n_planes)
    d = rng.standard_normal((n_planes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = t_true[anchor] + d * (place_radius * np.cbrt(rng.uniform(0.0, 1.0, size=n_planes)))[:, None]
    m = _truncated_geometric(rng, geom_p, m_max, n_planes)
    obs_v, obs_s = _nearest_observers(t_true, centres, m, obs_radius)
    npts = _loglog_counts(rng, pts_range[0], pts_range[1], obs_v.shape[0])
    s1, s2 = _cluster_sums(rng, centres, nrm, obs_v, obs_s, npts, r_true, t_true, sigma)
    init = _perturb(rng, r_true, t_true, math.radians(rot_bound_deg), trans_bound)
    return SumsScene(name or f"city-{n_scans}pose-{n_planes}vox", seed, obs_v, obs_s, npts, s1, s2, n_scans,
                     n_planes, _pack(r_true, t_true), init,
                     meta=dict(sigma=sigma, geom_p=geom_p, m_max=m_max, pts_range=pts_range))


def _window_part(rng, n_poses, n_planes, spacing, m_range, pts, sigma, offset, near):
    """One window with the tiny-scene law on a straight path: yaw uniform,
    planes centred within ``offset`` of a random anchor pose, each observed by
    m ~ U{m_range} distinct scans among the ``near`` poses nearest the anchor."""
    t_true = np.stack([spacing * np.arange(n_poses), np.zeros(n_poses), np.zeros(n_poses)], axis=1)
    r_true = _rz(rng.uniform(-math.pi, math.pi, size=n_poses))
    nrm = _unit_normals(rng, n_planes)
    anchor = rng.integers(0, n_poses, size=n_planes)
    d = rng.standard_normal((n_planes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = t_true[anchor] + d * rng.uniform(0.0, offset, size=n_planes)[:, None]
    nb = min(near, n_poses)
    m = np.minimum(rng.integers(m_range[0], m_range[1] + 1, size=n_planes), nb)
    lo = np.clip(anchor - nb // 2, 0, n_poses - nb)
    # m distinct offsets in [0, nb): the first m of a random permutation (argsort of uniforms)
    perm = np.argsort(rng.uniform(size=(n_planes, nb)), axis=1)
    take = np.arange(nb)[None, :] < m[:, None]
    cand = np.sort(np.where(take, perm, nb), axis=1)
    keep = cand < nb
    obs_s = (lo[:, None] + cand)[keep].astype(np.int32)
    obs_v = np.repeat(np.arange(n_planes, dtype=np.int32), keep.sum(axis=1))
    npts = np.full(obs_v.shape[0], pts, np.int64)
    s1, s2 = _cluster_sums(rng, centres, nrm, obs_v, obs_s, npts, r_true, t_true, sigma)
    return t_true, r_true, obs_v, obs_s, npts, s1, s2


def _window_job(args):
    seed, w, n_poses, n_planes, kw = args
    # window w draws from its own stream: Philox keyed by the seed, advanced
    # by (w + 1) jumps of 2^128 draws, so windows can be generated in parallel
    rng = np.random.Generator(np.random.Philox(key=int(seed)).jumped(w + 1))
    return _window_part(rng, n_poses, n_planes, **kw)


def batch_windows(seed: int = 4000, n_windows: int = 256, poses_range=(20, 400), vox_per_pose: int = 200,
                  vox_range=(5000, 80000), m_range=(3, 8), pts: int = 50, sigma: float = 0.02,
                  rot_bound_deg: float = 0.5, trans_bound: float = 0.05, spacing: float = 2.0,
                  offset: float = 30.0, near: int = 16, workers: int | None = None,
                  name: str | None = None, poses=None) -> SumsScene:
    """Batched workload: ``n_windows`` independent windows with poses per
    window log-uniform in ``poses_range`` (or the counts ``poses``, one per
    window, when given) and clip(vox_per_pose * N_w,
    vox_range) planes, each window with the tiny-scene law (3..8 observers,
    50 points, sigma = 2 cm, +-0.5 deg / +-5 cm) on a straight path with
    ``spacing`` metres between poses.  Scan and voxel ids are global; window w
    owns a contiguous scan range.  Windows are generated by up to ``workers``
    processes (default: min(16, cpu count)); the result does not depend on it."""
    import os
    rng = _rng(seed)
    Nw = _loglog_counts(rng, poses_range[0], poses_range[1], n_windows)
    if poses is not None:
        assert len(poses) == n_windows and min(poses) >= 1
        Nw = np.asarray(poses, dtype=Nw.dtype)
    Vw = np.clip(vox_per_pose * Nw, vox_range[0], vox_range[1])
    kw = dict(spacing=spacing, m_range=m_range, pts=pts, sigma=sigma, offset=offset, near=near)
    jobs = [(seed, w, int(Nw[w]), int(Vw[w]), kw) for w in range(n_windows)]
    workers = workers or min(16, os.cpu_count() or 1)
    if workers > 1 and n_windows > 1:
        with _pool(workers) as ex:
            parts = list(ex.map(_window_job, jobs, chunksize=1))
    else:
        parts = [_window_job(j) for j in jobs]
    s_off = np.concatenate([[0], np.cumsum(Nw)])
    v_off = np.concatenate([[0], np.cumsum(Vw)])
    t_true = np.concatenate([p[0] for p in parts])
    r_true = np.concatenate([p[1] for p in parts])
    init = _perturb(rng, r_true, t_true, math.radians(rot_bound_deg), trans_bound)
    sw = np.repeat(np.arange(n_windows, dtype=np.int32), Nw)
    vox = np.concatenate([p[2] + np.int32(v_off[w]) for w, p in enumerate(parts)])
    scan = np.concatenate([p[3] + np.int32(s_off[w]) for w, p in enumerate(parts)])
    return SumsScene(name or f"batch-{n_windows}win", seed, vox, scan, np.concatenate([p[4] for p in parts]),
                     np.concatenate([p[5] for p in parts]), np.concatenate([p[6] for p in parts]),
                     int(s_off[-1]), int(v_off[-1]), _pack(r_true, t_true), init, n_windows=n_windows,
                     scan_window=sw, meta=dict(poses=Nw.tolist(), voxels=Vw.tolist(), sigma=sigma))


def window_of(sc: SumsScene, w: int) -> SumsScene:
    """Window w of a batch as a problem of its own (scan and voxel ids rebased)."""
    s_lo = int(np.searchsorted(sc.scan_window, w, side="left"))
    s_hi = int(np.searchsorted(sc.scan_window, w, side="right"))
    sel = (sc.scan >= s_lo) & (sc.scan < s_hi)
    vox = sc.voxel[sel]
    v_lo, v_hi = int(vox.min()), int(vox.max()) + 1
    return SumsScene(f"{sc.name}/w{w}", sc.seed, (vox - v_lo).astype(np.int32),
                     (sc.scan[sel] - s_lo).astype(np.int32), sc.count[sel].copy(), sc.sum[sel].copy(),
                     sc.sumsq[sel].copy(), s_hi - s_lo, v_hi - v_lo, sc.poses_true[s_lo:s_hi].copy(),
                     sc.poses_init[s_lo:s_hi].copy(), meta=dict(window=w))


def request_scene(seed: int, n_poses: int, vox_per_pose: int = 400, **kw) -> SumsScene:
    """One served request: a single window of ``n_poses`` poses with about
    ``vox_per_pose`` planes per pose and the batched-window law."""
    rng = _rng(seed)
    t, r, ov, os_, npts, s1, s2 = _window_part(rng, n_poses, vox_per_pose * n_poses, kw.get("spacing", 2.0),
                                               kw.get("m_range", (3, 8)), kw.get("pts", 50),
                                               kw.get("sigma", 0.02), kw.get("offset", 30.0), kw.get("near", 16))
    init = _perturb(rng, r, t, math.radians(kw.get("rot_bound_deg", 0.5)), kw.get("trans_bound", 0.05))
    return SumsScene(f"request-{n_poses}pose", seed, ov, os_, npts, s1, s2, n_poses, vox_per_pose * n_poses,
                     _pack(r, t), init)


def _sweep_sums_job(args):
    seed, k, centres, nrm, obs_s, npts, r_true, t_true, sigma = args
    # chunk k draws from its own stream: Philox keyed by the seed, advanced by
    # (k + 1) jumps of 2^128 draws (the main stream is the unjumped one); its
    # planes arrive as one row per observation (plane index = row)
    rng = np.random.Generator(np.random.Philox(key=int(seed)).jumped(k + 1))
    local = np.arange(obs_s.shape[0], dtype=np.int64)
    return _cluster_sums(rng, centres, nrm, local, obs_s, npts, r_true, t_true, sigma, chunk=obs_s.shape[0])


def city_sweep_scene(n_scans: int, planes_per_pose: int = 500, seed: int = 5000, geom_p: float = 0.15,
                     m_max: int = 30, pts_range=(20, 1000), sigma: float = 0.03, rot_bound_deg: float = 1.0,
                     trans_bound: float = 0.10, place_radius: float = 40.0, obs_radius: float = 80.0,
                     chunk: int = 1 << 20, workers: int | None = None) -> SumsScene:
    """A member of the scaling sweep: the city law (``city_config``) with the
    loop grown in proportion to the pose count, so pose spacing (6.5 m),
    planes per pose and observers per plane stay fixed and the cluster count
    grows linearly with ``n_scans`` (2000 poses: a 5 km x 1 km loop).  The
    cluster statistics are drawn in chunks of ``chunk`` observations, each
    from its own jumped Philox stream, by up to ``workers`` processes
    (default: min(16, cpu count)); the result does not depend on it."""
    import os
    rng = _rng(seed)
    f = n_scans / 2000.0
    t_true, head = _city_trajectory(n_scans, width=5000.0 * f, height=1000.0 * f)
    r_true = _rz(head)
    n_planes = planes_per_pose * n_scans
    nrm = _unit_normals(rng, n_planes)
    anchor = rng.integers(0, n_scans, size=n_planes)
    d = rng.standard_normal((n_planes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = t_true[anchor] + d * (place_radius * np.cbrt(rng.uniform(0.0, 1.0, size=n_planes)))[:, None]
    m = _truncated_geometric(rng, geom_p, m_max, n_planes)
    obs_v, obs_s = _nearest_observers(t_true, centres, m, obs_radius)
    npts = _loglog_counts(rng, pts_range[0], pts_range[1], obs_v.shape[0])
    C = obs_v.shape[0]
    def jobs():
        for k, a in enumerate(range(0, C, chunk)):
            b = min(C, a + chunk)
            v = obs_v[a:b]
            yield (seed, k, centres[v], nrm[v], obs_s[a:b], npts[a:b], r_true, t_true, sigma)
    workers = workers or min(16, os.cpu_count() or 1)
    if workers > 1 and C > chunk:
        with _pool(workers) as ex:
            parts = list(ex.map(_sweep_sums_job, jobs(), chunksize=1))
    else:
        parts = [_sweep_sums_job(j) for j in jobs()]
    s1 = np.concatenate([p[0] for p in parts])
    s2 = np.concatenate([p[1] for p in parts])
    init = _perturb(rng, r_true, t_true, math.radians(rot_bound_deg), trans_bound)
    return SumsScene(f"city-sweep-{n_scans}pose-{n_planes}vox", seed, obs_v, obs_s, npts, s1, s2, n_scans,
                     n_planes, _pack(r_true, t_true), init,
                     meta=dict(sigma=sigma, geom_p=geom_p, m_max=m_max, pts_range=pts_range,
                               planes_per_pose=planes_per_pose))
