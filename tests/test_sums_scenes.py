"""CPU checks of the raw-sum scene generator (input synthesis only): the
clusters it draws have the statistics of the virtual point law it states."""
import numpy as np

import scenes.sums as ss


def _centred(sc):
    n = sc.count.astype(np.float64)
    mu = sc.sum / n[:, None]
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    S = np.empty((n.shape[0], 3, 3))
    for q, (i, j) in enumerate(iu):
        S[:, i, j] = S[:, j, i] = sc.sumsq[:, q] - n * mu[:, i] * mu[:, j]
    return n, mu, S


def test_request_scene_scatter_law():
    """Mean centred scatter over many clusters: eigenvalues (n - 1) * (1/12,
    1/12, sigma^2) in the plane frame, positive semi-definite throughout."""
    sc = ss.request_scene(seed=5, n_poses=30, vox_per_pose=60)
    n, mu, S = _centred(sc)
    ev = np.linalg.eigvalsh(S / (n - 1.0)[:, None, None])
    assert np.all(ev[:, 0] > 0)
    # the smallest eigenvalue is the normal spread sigma^2 = 4e-4 on average
    assert abs(np.mean(ev[:, 0]) / 4e-4 - 1.0) < 0.05
    # the in-plane ones average 1/12
    assert abs(np.mean(ev[:, 1:]) * 12.0 - 1.0) < 0.05


def test_clusters_lie_on_their_plane_at_the_true_poses():
    """Mapped by the true poses, the clusters of one voxel share one plane:
    normal spread of their centroids about the fitted plane is ~ sigma/sqrt(N)."""
    sc = ss.request_scene(seed=7, n_poses=20, vox_per_pose=20)
    n, mu, _ = _centred(sc)
    R = sc.poses_true[:, :9].reshape(-1, 3, 3)
    t = sc.poses_true[:, 9:]
    xw = np.einsum("kij,kj->ki", R[sc.scan], mu) + t[sc.scan]
    worst = 0.0
    for v in np.unique(sc.voxel):
        sel = sc.voxel == v
        if sel.sum() < 4:
            continue
        x = xw[sel] - xw[sel].mean(0)
        _, s, _ = np.linalg.svd(x, full_matrices=False)
        worst = max(worst, s[-1] / np.sqrt(sel.sum()))
    assert worst < 0.02 * 4 / np.sqrt(50)


def test_batch_windows_are_disjoint_and_parallel_generation_is_exact():
    a = ss.batch_windows(seed=11, n_windows=5, poses_range=(6, 20), vox_per_pose=20, vox_range=(50, 300),
                         workers=1)
    b = ss.batch_windows(seed=11, n_windows=5, poses_range=(6, 20), vox_per_pose=20, vox_range=(50, 300),
                         workers=3)
    for f in ("voxel", "scan", "count", "sum", "sumsq", "poses_init", "scan_window"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert np.all(np.diff(a.scan_window) >= 0)
    # every voxel's observers lie in one window
    wv = a.scan_window[a.scan]
    for v in np.unique(a.voxel):
        assert np.unique(wv[a.voxel == v]).size == 1
    # window_of rebases ids and keeps the clusters
    tot = 0
    for w in range(a.n_windows):
        sw = ss.window_of(a, w)
        assert sw.scan.min() >= 0 and sw.scan.max() < sw.n_scans
        assert sw.voxel.min() >= 0 and sw.voxel.max() < sw.n_voxels
        tot += sw.n_clusters
    assert tot == a.n_clusters


def test_city_sweep_parallel_generation_is_exact_and_scales_linearly():
    """The scaling-sweep scenes do not depend on the number of generator
    processes, keep the pose spacing of the 2000-pose city loop, and grow
    their cluster count in proportion to the pose count."""
    a = ss.city_sweep_scene(400, planes_per_pose=60, chunk=1 << 13, workers=3)
    b = ss.city_sweep_scene(400, planes_per_pose=60, chunk=1 << 13, workers=1)
    for k in ("voxel", "scan", "count", "sum", "sumsq", "poses_true", "poses_init"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    c = ss.city_sweep_scene(800, planes_per_pose=60, chunk=1 << 13, workers=2)
    step = lambda sc: np.median(np.linalg.norm(np.diff(sc.poses_true[:, 9:], axis=0), axis=1))
    # 13 km of route (12 km loop + 1 km cross street) for 2000 poses: 6.5 m
    # between poses at every size
    assert abs(step(a) - 6.5) < 0.05 and abs(step(c) - 6.5) < 0.05
    assert abs(c.n_clusters / a.n_clusters - 2.0) < 0.1
    # every cluster's scatter is positive semi-definite in the scan frame
    n, mu, S = _centred(c)
    assert np.all(np.linalg.eigvalsh(S)[:, 0] > -1e-9 * np.abs(S).max(axis=(1, 2)))


def test_sweep_scene_does_not_depend_on_the_worker_count():
    """The scaling-sweep generator draws each chunk from its own stream and
    hands every worker its chunk's data: one process and three give the same
    clusters."""
    a = ss.city_sweep_scene(40, planes_per_pose=20, chunk=500, workers=1)
    b = ss.city_sweep_scene(40, planes_per_pose=20, chunk=500, workers=3)
    assert a.n_clusters > 4 * 500
    for f in ("voxel", "scan", "count", "sum", "sumsq", "poses_init"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
