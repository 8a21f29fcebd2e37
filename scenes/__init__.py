"""Seeded synthetic LiDAR bundle-adjustment scenes.

This module only *synthesises inputs*: scan poses, planar patches and raw
body-frame points with their scan and voxel labels.  It performs none of the
method's arithmetic (no point clusters, no covariances, no eigenvalues, no
derivatives); both the CPU oracle and the GPU path consume the same arrays it
returns and build their own clusters from them.

Scene law (stands in for the paper's HeLiPR / MulRan / MaRS-LVIG sequences,
which are not available; Sec. VI-A describes those datasets):

* plane normals uniform on the sphere, a 1 m x 1 m square patch per plane,
  points uniform on the patch plus N(0, sigma^2) noise along the normal;
* every plane is one voxel, observed by ``m`` scans; each (voxel, scan)
  observation contributes ``n`` points expressed in that scan's body frame
  with the true pose, ``p = R^T (x - t)``;
* true orientations are yaw-only ``Rz(psi)``; the initial estimate is the
  truth perturbed by a rotation of uniform +-rot_bound per axis (left
  multiplied) and a translation of uniform +-trans_bound per axis.

All randomness comes from numpy's Philox4x32-10 counter-based generator
(Salmon et al., SC'11), keyed by the seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Scene:
    """Raw synthetic scene.  Points are SoA, float64, in scan body frames."""

    name: str
    seed: int
    x: np.ndarray            # (P,) float64
    y: np.ndarray            # (P,) float64
    z: np.ndarray            # (P,) float64
    scan: np.ndarray         # (P,) int32, 0 <= scan < n_scans
    voxel: np.ndarray        # (P,) int32, 0 <= voxel < n_voxels
    n_scans: int
    n_voxels: int
    poses_true: np.ndarray   # (n_scans, 12) float64: R row-major, then t
    poses_init: np.ndarray   # (n_scans, 12) float64
    n_clusters: int          # number of distinct (voxel, scan) observations
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.x.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def _rz(psi: np.ndarray) -> np.ndarray:
    c, s = np.cos(psi), np.sin(psi)
    r = np.zeros((psi.shape[0], 3, 3))
    r[:, 0, 0] = c
    r[:, 0, 1] = -s
    r[:, 1, 0] = s
    r[:, 1, 1] = c
    r[:, 2, 2] = 1.0
    return r


def _quat_rot(omega: np.ndarray) -> np.ndarray:
    """Rotation by angle |omega| about omega/|omega|, built from a unit
    quaternion (scene synthesis only)."""
    th = np.linalg.norm(omega, axis=1)
    half = 0.5 * th
    with np.errstate(invalid="ignore", divide="ignore"):
        k = np.where(th > 0, np.sin(half) / np.where(th > 0, th, 1.0), 0.5)
    qw = np.cos(half)
    qx, qy, qz = (omega * k[:, None]).T
    r = np.empty((omega.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    r[:, 0, 1] = 2 * (qx * qy - qz * qw)
    r[:, 0, 2] = 2 * (qx * qz + qy * qw)
    r[:, 1, 0] = 2 * (qx * qy + qz * qw)
    r[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    r[:, 1, 2] = 2 * (qy * qz - qx * qw)
    r[:, 2, 0] = 2 * (qx * qz - qy * qw)
    r[:, 2, 1] = 2 * (qy * qz + qx * qw)
    r[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return r


def _pack(r: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([r.reshape(-1, 9), t], axis=1).astype(np.float64)


def _unit_normals(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _inplane_basis(nrm):
    # any vector not parallel to n, Gram-Schmidt
    a = np.where(np.abs(nrm[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = a - (a * nrm).sum(1, keepdims=True) * nrm
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nrm, e1)
    return e1, e2


def _perturb(rng, r_true, t_true, rot_bound, trans_bound):
    n = r_true.shape[0]
    om = rng.uniform(-rot_bound, rot_bound, size=(n, 3))
    tau = rng.uniform(-trans_bound, trans_bound, size=(n, 3))
    r0 = np.einsum("nij,njk->nik", _quat_rot(om), r_true)
    return _pack(r0, t_true + tau)


def _emit_points(rng, centres, normals, obs_voxel, obs_scan, obs_npts, r_true, t_true,
                 sigma, patch=1.0, chunk=50_000):
    """Sample the raw points of every (voxel, scan) observation.

    Observations are emitted in the given order, each one's points contiguous.
    A point is x = c + a e1 + b e2 + eps n in the world (a, b uniform on the
    patch, eps ~ N(0, sigma^2)); its body-frame coordinates R^T (x - t) are
    assembled from the observation's body-frame patch basis.
    """
    e1, e2 = _inplane_basis(normals)
    rt = np.transpose(r_true, (0, 2, 1))            # R^T per scan
    ro = rt[obs_scan]                               # (nobs, 3, 3)
    o = np.einsum("nij,nj->ni", ro, centres[obs_voxel] - t_true[obs_scan])
    f1 = np.einsum("nij,nj->ni", ro, e1[obs_voxel])
    f2 = np.einsum("nij,nj->ni", ro, e2[obs_voxel])
    f3 = np.einsum("nij,nj->ni", ro, normals[obs_voxel])
    total = int(obs_npts.sum())
    out = [np.empty(total), np.empty(total), np.empty(total)]
    scan = np.repeat(obs_scan.astype(np.int32), obs_npts)
    voxel = np.repeat(obs_voxel.astype(np.int32), obs_npts)
    offs = np.concatenate([[0], np.cumsum(obs_npts)])
    nobs = obs_voxel.shape[0]
    for a in range(0, nobs, chunk):
        b = min(nobs, a + chunk)
        cnt = obs_npts[a:b]
        p0, p1 = int(offs[a]), int(offs[b])
        k = p1 - p0
        ua = rng.uniform(-0.5 * patch, 0.5 * patch, size=k)
        ub = rng.uniform(-0.5 * patch, 0.5 * patch, size=k)
        eps = rng.standard_normal(k)
        eps *= sigma
        tmp = np.empty(k)
        for d in range(3):
            dst = out[d][p0:p1]
            dst[:] = np.repeat(o[a:b, d], cnt)
            np.multiply(ua, np.repeat(f1[a:b, d], cnt), out=tmp)
            dst += tmp
            np.multiply(ub, np.repeat(f2[a:b, d], cnt), out=tmp)
            dst += tmp
            np.multiply(eps, np.repeat(f3[a:b, d], cnt), out=tmp)
            dst += tmp
    return out[0], out[1], out[2], scan, voxel


def _shuffle_points(rng, sc_arrays):
    perm = rng.permutation(sc_arrays[0].shape[0])
    return [a[perm] for a in sc_arrays]


def small_scene(seed: int = 1000, n_scans: int = 10, n_planes: int = 200, path_len: float = 20.0,
                offset_range: float = 30.0, m_range=(3, 8), pts_per_obs=(50, 50), sigma: float = 0.02,
                rot_bound_deg: float = 0.5, trans_bound: float = 0.05, shuffle: bool = False,
                name: str = "tiny") -> Scene:
    """Tiny scene: ``n_scans`` poses on a straight path of ``path_len`` metres,
    ``n_planes`` planes with offsets uniform in +-offset_range (patch centred at
    the foot point d*n), each seen by m ~ U{m_range} distinct random scans with
    ``pts_per_obs`` points (uniform integer range) per observation."""
    rng = _rng(seed)
    if n_scans > 1:
        tx = path_len * np.arange(n_scans) / (n_scans - 1)
    else:
        tx = np.zeros(1)
    t_true = np.stack([tx, np.zeros(n_scans), np.zeros(n_scans)], axis=1)
    r_true = _rz(rng.uniform(-math.pi, math.pi, size=n_scans))
    nrm = _unit_normals(rng, n_planes)
    off = rng.uniform(-offset_range, offset_range, size=n_planes)
    centres = nrm * off[:, None]
    lo, hi = m_range
    m = rng.integers(lo, hi + 1, size=n_planes)
    m = np.minimum(m, n_scans)
    obs_v, obs_s = [], []
    for i in range(n_planes):
        sc = np.sort(rng.choice(n_scans, size=int(m[i]), replace=False))
        obs_v.append(np.full(sc.shape[0], i, np.int32))
        obs_s.append(sc.astype(np.int32))
    obs_v = np.concatenate(obs_v)
    obs_s = np.concatenate(obs_s)
    npts = rng.integers(pts_per_obs[0], pts_per_obs[1] + 1, size=obs_v.shape[0])
    x, y, z, scan, voxel = _emit_points(rng, centres, nrm, obs_v, obs_s, npts, r_true, t_true, sigma)
    init = _perturb(rng, r_true, t_true, math.radians(rot_bound_deg), trans_bound)
    if shuffle:
        x, y, z, scan, voxel = _shuffle_points(rng, [x, y, z, scan, voxel])
    return Scene(name=name, seed=seed, x=x, y=y, z=z, scan=scan, voxel=voxel,
                 n_scans=n_scans, n_voxels=n_planes, poses_true=_pack(r_true, t_true),
                 poses_init=init, n_clusters=int(obs_v.shape[0]),
                 meta=dict(sigma=sigma, rot_bound_deg=rot_bound_deg, trans_bound=trans_bound))


def tiny_config(seed: int = 1000, sigma: float = 0.02, shuffle: bool = False) -> Scene:
    """The tiny plain-FP64 workload: 10 poses on a 20 m path, 200 planes with
    offsets in +-30 m, 3..8 observing scans per plane, 50 points per
    observation, N(0, sigma) normal noise, +-0.5 deg / +-5 cm perturbation."""
    return small_scene(seed=seed, sigma=sigma, shuffle=shuffle, name="tiny-10pose-200vox")


def _figure_eight(n_poses: int, length: float):
    """Poses every length/n_poses metres along two tangent circles that cross
    at the origin (a closed figure-eight, giving loop closures at the
    crossing)."""
    r = length / (4.0 * math.pi)
    s = np.arange(n_poses) * (length / n_poses)
    half = length / 2.0
    pts = np.zeros((n_poses, 3))
    head = np.zeros(n_poses)
    for k, sk in enumerate(s):
        if sk < half:
            a = sk / r                      # first circle, centre (-r, 0), ccw
            pts[k, 0] = -r + r * math.cos(a)
            pts[k, 1] = r * math.sin(a)
            head[k] = a + math.pi / 2
        else:
            a = (sk - half) / r             # second circle, centre (+r, 0), cw
            pts[k, 0] = r - r * math.cos(a)
            pts[k, 1] = r * math.sin(a)
            head[k] = math.pi / 2 - a
    return pts, head


def window_scene(seed: int = 2000, n_scans: int = 500, n_planes: int = 200_000, length: float = 2000.0,
                 place_radius: float = 40.0, obs_radius: float = 80.0, geom_p: float = 0.25,
                 m_max: int = 20, pts_range=(20, 500), sigma: float = 0.03,
                 rot_bound_deg: float = 1.0, trans_bound: float = 0.10, shuffle: bool = False,
                 name: str | None = None) -> Scene:
    """Single-window workload: ``n_scans`` poses on a closed figure-eight of
    ``length`` metres; every plane is centred within ``place_radius`` of a
    random anchor pose and observed by its m nearest poses within
    ``obs_radius`` (m ~ geometric(p) truncated to [1, m_max]); points per
    observation log-uniform in ``pts_range``."""
    rng = _rng(seed)
    t_true, head = _figure_eight(n_scans, length)
    r_true = _rz(head)
    nrm = _unit_normals(rng, n_planes)
    anchor = rng.integers(0, n_scans, size=n_planes)
    d = rng.standard_normal((n_planes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = place_radius * np.cbrt(rng.uniform(0.0, 1.0, size=n_planes))
    centres = t_true[anchor] + d * rad[:, None]
    # truncated geometric on [1, m_max]
    k = np.arange(1, m_max + 1)
    pk = (1 - geom_p) ** (k - 1) * geom_p
    pk /= pk.sum()
    m = rng.choice(k, size=n_planes, p=pk)
    # the m nearest poses within obs_radius (at least the nearest one)
    from scipy.spatial import cKDTree
    tree = cKDTree(t_true)
    kq = min(m_max, n_scans)
    dist, idx = tree.query(centres, k=kq, distance_upper_bound=obs_radius)
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
    lo, hi = pts_range
    npts = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=obs_v.shape[0]))).astype(np.int64)
    npts = np.clip(npts, lo, hi)
    x, y, z, scan, voxel = _emit_points(rng, centres, nrm, obs_v, obs_s, npts, r_true, t_true, sigma)
    init = _perturb(rng, r_true, t_true, math.radians(rot_bound_deg), trans_bound)
    if shuffle:
        x, y, z, scan, voxel = _shuffle_points(rng, [x, y, z, scan, voxel])
    if name is None:
        name = f"window-{n_scans}pose-{n_planes}vox"
    return Scene(name=name, seed=seed, x=x, y=y, z=z, scan=scan, voxel=voxel,
                 n_scans=n_scans, n_voxels=n_planes, poses_true=_pack(r_true, t_true),
                 poses_init=init, n_clusters=int(obs_v.shape[0]),
                 meta=dict(sigma=sigma, rot_bound_deg=rot_bound_deg, trans_bound=trans_bound,
                           geom_p=geom_p, m_max=m_max, pts_range=pts_range))


def window_config(seed: int = 2000, shuffle: bool = False) -> Scene:
    """The single-window FP64 workload: 500 poses on a 2 km figure-eight,
    200k planar voxels, 1..20 observing scans (geometric p = 0.25),
    20..500 points per observation (log-uniform), N(0, 0.03 m) noise,
    +-1 deg / +-10 cm perturbation."""
    return window_scene(seed=seed, shuffle=shuffle, name="window-500pose-200kvox")


def scaled_window(seed: int = 2001, n_scans: int = 60, n_planes: int = 3000, pts_range=(20, 60),
                  shuffle: bool = False) -> Scene:
    """A small scene with the single-window law (geometric observer counts,
    log-uniform point counts, loop closures) for fast tests."""
    length = 4.0 * n_scans
    return window_scene(seed=seed, n_scans=n_scans, n_planes=n_planes, length=length,
                        place_radius=min(40.0, length / 8), obs_radius=min(80.0, length / 4),
                        pts_range=pts_range, shuffle=shuffle,
                        name=f"scaled-window-{n_scans}pose-{n_planes}vox")


def rigid_transform_poses(poses: np.ndarray, rot: np.ndarray, trans: np.ndarray) -> np.ndarray:
    """Left-multiply every pose by one global rigid motion G = (rot, trans):
    R_j -> rot R_j, t_j -> rot t_j + trans.  Used to build gauge-invariance
    test inputs."""
    r = poses[:, :9].reshape(-1, 3, 3)
    t = poses[:, 9:]
    r2 = np.einsum("ij,njk->nik", rot, r)
    t2 = t @ rot.T + trans
    return _pack(r2, t2)
