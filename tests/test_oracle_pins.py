"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: brute force over
raw points, LAPACK eigen-solvers, finite differences, closed forms, gauge
invariance and the majorization chain.  None needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers
def world_points(sc, poses):
    R = poses[:, :9].reshape(-1, 3, 3)
    t = poses[:, 9:]
    p = np.stack([sc.x, sc.y, sc.z], axis=1)
    Rs = R[sc.scan]
    return np.einsum("nij,nj->ni", Rs, p) + t[sc.scan]


def brute_voxel_cov(sc, poses, dtype=np.float64):
    """Covariance of every voxel's transformed raw points (Eq. 1), by brute force."""
    q = world_points(sc, poses).astype(dtype)
    out = np.zeros((sc.n_voxels, 3, 3), dtype=dtype)
    cnt = np.zeros(sc.n_voxels)
    for v in range(sc.n_voxels):
        sel = sc.voxel == v
        qq = q[sel]
        cnt[v] = qq.shape[0]
        if qq.shape[0] == 0:
            continue
        d = qq - qq.mean(axis=0)
        out[v] = d.T @ d / qq.shape[0]
    return out, cnt


def sym6_to_full(a6):
    a = np.empty(a6.shape[:-1] + (3, 3))
    a[..., 0, 0] = a6[..., 0]; a[..., 0, 1] = a6[..., 1]; a[..., 0, 2] = a6[..., 2]
    a[..., 1, 0] = a6[..., 1]; a[..., 1, 1] = a6[..., 3]; a[..., 1, 2] = a6[..., 4]
    a[..., 2, 0] = a6[..., 2]; a[..., 2, 1] = a6[..., 4]; a[..., 2, 2] = a6[..., 5]
    return a


def dense_mm(H_mm):
    n = H_mm.shape[0]
    D = np.zeros((6 * n, 6 * n))
    for j in range(n):
        D[6 * j:6 * j + 6, 6 * j:6 * j + 6] = H_mm[j]
    return D


def gauge_basis(poses):
    """6N x 6 basis of the global rigid motions in the chart (Exp(phi)R, t+dt):
    a world rotation eps moves pose j by [eps; eps x t_j], a world translation
    by [0; d]."""
    n = poses.shape[0]
    V = np.zeros((6 * n, 6))
    for j in range(n):
        t = poses[j, 9:]
        V[6 * j:6 * j + 3, 0:3] = np.eye(3)
        tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
        V[6 * j + 3:6 * j + 6, 0:3] = -tx
        V[6 * j + 3:6 * j + 6, 3:6] = np.eye(3)
    return V


def step(orc, poses, k, h):
    dx = np.zeros(6 * poses.shape[0])
    dx[k] = h
    return orc.apply_increment(poses, dx)


def small(seed=7, sigma=0.02, **kw):
    kw.setdefault("n_scans", 4)
    kw.setdefault("n_planes", 30)
    kw.setdefault("m_range", (2, 4))
    kw.setdefault("pts_per_obs", (8, 20))
    kw.setdefault("path_len", 6.0)
    kw.setdefault("offset_range", 6.0)
    return scenes.small_scene(seed=seed, sigma=sigma, **kw)


@pytest.fixture(scope="module")
def tiny(orc):
    sc = scenes.tiny_config(seed=1000, shuffle=True)
    return sc, orc.scene_clusters(sc)


# ---------------------------------------------------------------- P1, P2: clusters and covariance
def test_clusters_match_bruteforce(orc, tiny):
    sc, cl = tiny
    assert cl.C == sc.n_clusters
    p = np.stack([sc.x, sc.y, sc.z], axis=1)
    for c in range(0, cl.C, 37):
        sel = (sc.voxel == cl.vox[c]) & (sc.scan == cl.scan[c])
        pts = p[sel]
        assert pts.shape[0] == cl.n[c]
        mu = pts.mean(axis=0)
        d = pts - mu
        S = d.T @ d
        assert np.allclose(cl.mu[c], mu, rtol=0, atol=1e-13 * (1 + np.abs(mu).max()))
        Sf = sym6_to_full(cl.S[c])
        assert np.abs(Sf - S).max() <= 1e-12 * np.abs(S).max()


def test_voxel_covariance_bruteforce(orc, tiny):
    sc, cl = tiny
    st = orc.voxel_stats(cl, sc.poses_init)
    cov, cnt = brute_voxel_cov(sc, sc.poses_init)
    A = sym6_to_full(st["A"])
    assert np.array_equal(st["N"], cnt)
    err = np.abs(A - cov).max(axis=(1, 2)) / np.abs(cov).max(axis=(1, 2))
    assert err.max() <= 1e-12


def test_raw_sum_form_matches_centred(orc, tiny):
    """Eq. 2's raw-sum interchange, centred once in binary128, equals the
    two-pass centred clusters up to the double rounding of the raw sums."""
    sc, cl = tiny
    vox, scan, n, s1, s2 = orc.points_to_raw_sums(sc.x, sc.y, sc.z, sc.scan, sc.voxel)
    assert np.array_equal(vox, cl.vox) and np.array_equal(scan, cl.scan) and np.array_equal(n, cl.n)
    mu, S = orc.center_raw_sums(n, s1, s2)
    assert np.abs(mu - cl.mu).max() <= 1e-13
    # raw second moments at |p| ~ 30 m keep ~1e-16 * N * 900 absolute accuracy
    bound = 4e-16 * n[:, None] * np.max(np.abs(cl.mu), axis=1, keepdims=True) ** 2 + 1e-15
    assert np.all(np.abs(S - cl.S) <= bound)


# ---------------------------------------------------------------- P3: eigen
def test_eig3_against_lapack(orc):
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((3, 3)) for _ in range(200)]
    mats = [m + m.T for m in mats]
    mats += [np.diag([3.0, 1.0, 2.0]), np.diag([1.0, 1.0, 2.0]), np.eye(3), np.zeros((3, 3)),
             np.array([[2.0, 1e-20, 0], [1e-20, 2.0, 0], [0, 0, 1.0]])]
    # planar-like covariance with tiny smallest eigenvalue
    Q = Rotation.from_rotvec([0.3, -0.2, 0.7]).as_matrix()
    mats.append(Q @ np.diag([1e-6, 0.08, 0.09]) @ Q.T)
    for m in mats:
        a6 = np.array([m[0, 0], m[0, 1], m[0, 2], m[1, 1], m[1, 2], m[2, 2]])
        lam, U = orc.eig3(a6)
        ref = np.linalg.eigvalsh(m)
        nrm = max(np.abs(ref).max(), 1e-300)
        assert np.abs(lam - ref).max() <= 1e-14 * nrm + 1e-300
        assert np.abs(U.T @ U - np.eye(3)).max() <= 1e-14
        assert np.abs(m @ U - U * lam).max() <= 4e-15 * nrm + 1e-300


# ---------------------------------------------------------------- P4: zero residual
def test_zero_residual_noise_free_truth(orc):
    sc = scenes.tiny_config(seed=1001, sigma=0.0)
    cl = orc.scene_clusters(sc)
    c = orc.cost(cl, sc.poses_true)
    st = orc.voxel_stats(cl, sc.poses_true)
    trace = st["A"][:, [0, 3, 5]].sum()
    assert abs(c) <= 1e-13 * trace
    assert orc.cost(cl, sc.poses_init) > 1e3 * abs(c)


# ---------------------------------------------------------------- P5: gauge invariance of the cost
@pytest.mark.parametrize("shift", [0.0, 10.0, 1000.0])
def test_cost_invariance_global_rigid(orc, tiny, shift):
    sc, cl = tiny
    rot = Rotation.from_rotvec([0.4, -1.1, 0.25]).as_matrix()
    trans = np.array([shift, -0.5 * shift, 0.3 * shift])
    P2 = scenes.rigid_transform_poses(sc.poses_init, rot, trans)
    c1 = orc.cost(cl, sc.poses_init)
    c2 = orc.cost(cl, P2)
    # at a 1 km offset the world coordinates themselves carry ~1e-13 m rounding
    tol = 1e-12 if shift <= 10 else 2e-11
    assert abs(c2 - c1) <= tol * c1


# ---------------------------------------------------------------- P6: surrogate (Eq. 3)
def eq3_literal(sc, poses, poses_l):
    """Eq. 3 exactly as printed, from raw points, in extended precision:
    sum_j [u^T P_ij u / N_i - 4 z u^T v_ij / N_i^2] + 4 z^2 / N_i^2 with
    u = u_min at T_l (LAPACK) and z = 1/2 sum_j u^T v_ij(T_l)."""
    ld = np.longdouble
    q = world_points(sc, poses).astype(ld)
    ql = world_points(sc, poses_l).astype(ld)
    covl, _ = brute_voxel_cov(sc, poses_l)
    total = ld(0)
    for v in range(sc.n_voxels):
        sel = sc.voxel == v
        if not sel.any():
            continue
        w, U = np.linalg.eigh(covl[v])
        u = U[:, 0].astype(ld)
        Ni = ld(sel.sum())
        z = ld(0.5) * (ql[sel] @ u).sum()
        acc = ld(0)
        for j in np.unique(sc.scan[sel]):
            s2 = sel & (sc.scan == j)
            qj = q[s2]
            Pij = qj.T @ qj
            vij = qj.sum(axis=0)
            acc += (u @ Pij @ u) / Ni - ld(4) * z / Ni ** 2 * (u @ vij)
        total += acc + ld(4) * z * z / Ni ** 2
    return float(total)


def test_surrogate_equals_eq3_literal(orc):
    sc = small(seed=11)
    cl = orc.scene_clusters(sc)
    Tl = sc.poses_init
    rng = np.random.default_rng(5)
    for trial in range(3):
        dx = rng.uniform(-0.01, 0.01, size=6 * sc.n_scans)
        T = orc.apply_increment(Tl, dx)
        lit = eq3_literal(sc, T, Tl)
        mine = orc.majorizer(0, cl, T, Tl)
        assert abs(mine - lit) <= 1e-12 * abs(lit)


def test_majorization_chain(orc, tiny):
    sc, cl = tiny
    Tl = sc.poses_init
    c_l = orc.cost(cl, Tl)
    assert abs(orc.majorizer(0, cl, Tl, Tl) - c_l) <= 1e-13 * c_l
    assert abs(orc.majorizer(1, cl, Tl, Tl) - c_l) <= 1e-13 * c_l
    rng = np.random.default_rng(9)
    for trial in range(10):
        dx = rng.uniform(-0.02, 0.02, size=6 * sc.n_scans)
        T = orc.apply_increment(Tl, dx)
        cm = orc.majorizer(0, cl, T, Tl)
        cc = orc.majorizer(1, cl, T, Tl)
        c = orc.cost(cl, T)
        assert cm >= cc - 1e-13 * cm
        assert cc >= c - 1e-13 * cc


# ---------------------------------------------------------------- chart
def test_so3_exp_against_library(orc):
    rng = np.random.default_rng(1)
    vecs = [rng.standard_normal(3) * s for s in (1e-12, 1e-9, 1e-7, 1e-4, 0.1, 1.0, 3.0)]
    vecs.append(np.zeros(3))
    for v in vecs:
        R = orc.so3_exp(v)
        ref = Rotation.from_rotvec(v).as_matrix()
        assert np.abs(R - ref).max() <= 2e-16 * 8


# ---------------------------------------------------------------- P7: gradient
@pytest.mark.parametrize("seed", [21, 22])
def test_gradient_finite_difference(orc, seed):
    sc = small(seed=seed)
    cl = orc.scene_clusters(sc)
    T = sc.poses_init
    c, g, H, _ = orc.evaluate(orc.MM, cl, T)
    h = 1e-5
    fd = np.empty_like(g)
    for k in range(g.shape[0]):
        cp1 = orc.cost(cl, step(orc, T, k, h)); cm1 = orc.cost(cl, step(orc, T, k, -h))
        cp2 = orc.cost(cl, step(orc, T, k, 2 * h)); cm2 = orc.cost(cl, step(orc, T, k, -2 * h))
        fd[k] = (-cp2 + 8 * cp1 - 8 * cm1 + cm2) / (12 * h)
    assert np.linalg.norm(fd - g) <= 1e-7 * np.linalg.norm(g)
    # the gradient is the same in every mode (majorizers touch c at T_l)
    for mode in (orc.COUPLED, orc.EXACT):
        _, g2, _, _ = orc.evaluate(mode, cl, T)
        assert np.array_equal(g, g2)


# ---------------------------------------------------------------- P8, P9: Hessians
def fd_hessian(f, T, n, orc, h=1e-4):
    D = 6 * n
    Hf = np.empty((D, D))
    for a in range(D):
        for b in range(a, D):
            def at(sa, sb):
                dx = np.zeros(D)
                dx[a] += sa * h
                dx[b] += sb * h
                return f(orc.apply_increment(T, dx))
            val = (at(1, 1) - at(1, -1) - at(-1, 1) + at(-1, -1)) / (4 * h * h)
            Hf[a, b] = Hf[b, a] = val
    return Hf


@pytest.fixture(scope="module")
def hess_scene(orc):
    sc = small(seed=31, n_scans=3, n_planes=16)
    cl = orc.scene_clusters(sc)
    return sc, cl


def test_mm_hessian_finite_difference(orc, hess_scene):
    sc, cl = hess_scene
    T = sc.poses_init
    _, g, Hmm, _ = orc.evaluate(orc.MM, cl, T)
    Hfd = fd_hessian(lambda P: orc.majorizer(0, cl, P, T), T, sc.n_scans, orc)
    Hd = dense_mm(Hmm)
    assert np.linalg.norm(Hfd - Hd) <= 1e-6 * np.linalg.norm(Hd)
    # the surrogate separates over scans: off-diagonal pose blocks vanish
    for j in range(sc.n_scans):
        for k in range(sc.n_scans):
            if j != k:
                assert np.abs(Hfd[6 * j:6 * j + 6, 6 * k:6 * k + 6]).max() <= 1e-6 * np.abs(Hd).max()
    for j in range(sc.n_scans):
        assert np.abs(Hmm[j] - Hmm[j].T).max() <= 1e-14 * np.abs(Hmm[j]).max()


def test_coupled_hessian_finite_difference(orc, hess_scene):
    sc, cl = hess_scene
    T = sc.poses_init
    _, _, Hc, _ = orc.evaluate(orc.COUPLED, cl, T)
    Hfd = fd_hessian(lambda P: orc.majorizer(1, cl, P, T), T, sc.n_scans, orc)
    assert np.linalg.norm(Hfd - Hc) <= 1e-6 * np.linalg.norm(Hc)
    assert np.abs(Hc - Hc.T).max() <= 1e-14 * np.abs(Hc).max()


def test_exact_hessian_finite_difference_of_gradient(orc, hess_scene):
    sc, cl = hess_scene
    T = sc.poses_init
    _, g, He, nd = orc.evaluate(orc.EXACT, cl, T)
    assert nd == 0
    D = g.shape[0]
    h = 1e-6
    Hfd = np.empty((D, D))
    for k in range(D):
        _, gp, _, _ = orc.evaluate(orc.MM, cl, step(orc, T, k, h))
        _, gm, _, _ = orc.evaluate(orc.MM, cl, step(orc, T, k, -h))
        Hfd[:, k] = (gp - gm) / (2 * h)
    # the chart's Hessian of c is symmetric only at first order in the step;
    # compare with the symmetrised finite difference
    Hfd = 0.5 * (Hfd + Hfd.T)
    assert np.linalg.norm(Hfd - He) <= 1e-6 * np.linalg.norm(He)


def test_hessian_ordering(orc, tiny):
    """H_MM >= H_C >= H_E at T_l: the majorizers are tangent from above."""
    sc, cl = tiny
    T = sc.poses_init
    _, _, Hmm, _ = orc.evaluate(orc.MM, cl, T)
    _, _, Hc, _ = orc.evaluate(orc.COUPLED, cl, T)
    _, _, He, _ = orc.evaluate(orc.EXACT, cl, T)
    Hm = dense_mm(Hmm)
    scale = np.abs(Hm).max()
    assert np.linalg.eigvalsh(Hm - Hc).min() >= -1e-12 * scale
    assert np.linalg.eigvalsh(Hc - He).min() >= -1e-12 * scale


# ---------------------------------------------------------------- P10: gauge
def test_gauge_gradient_orthogonal(orc, tiny):
    sc, cl = tiny
    for T in (sc.poses_init, sc.poses_true):
        _, g, Hc, _ = orc.evaluate(orc.COUPLED, cl, T)
        V = gauge_basis(T)
        assert np.abs(V.T @ g).max() <= 1e-12 * np.abs(g).sum()
        # global translations are an exact null space of H_C at any poses
        Vt = V[:, 3:]
        assert np.abs(Hc @ Vt).max() <= 1e-12 * np.abs(Hc).max()


def test_gauge_null_space_exact_hessian(orc):
    sc = scenes.tiny_config(seed=1002, sigma=0.0)
    cl = orc.scene_clusters(sc)
    T = sc.poses_true
    _, g, He, _ = orc.evaluate(orc.EXACT, cl, T)
    V = gauge_basis(T)
    Vq, _ = np.linalg.qr(V)
    assert np.linalg.norm(He @ Vq) <= 1e-11 * np.linalg.norm(He)
    ev = np.linalg.eigvalsh(He)
    lam_max = np.abs(ev).max()
    small_ev = np.sort(np.abs(ev))
    assert small_ev[5] <= 1e-12 * lam_max          # six gauge directions
    assert small_ev[6] >= 1e-8 * lam_max           # and no seventh
    # MM is anchored by the frozen planes: positive definite
    _, _, Hmm, _ = orc.evaluate(orc.MM, cl, T)
    assert min(np.linalg.eigvalsh(b).min() for b in Hmm) > 0


# ---------------------------------------------------------------- P11: single-scan voxels
def test_single_scan_voxels(orc):
    sc = small(seed=41, m_range=(1, 1))
    cl = orc.scene_clusters(sc)
    T = sc.poses_init
    _, g, Hmm, _ = orc.evaluate(orc.MM, cl, T)
    _, _, He, _ = orc.evaluate(orc.EXACT, cl, T)
    assert np.abs(g).max() <= 1e-13
    assert np.abs(He).max() <= 1e-12 * max(1.0, np.abs(dense_mm(Hmm)).max())
    assert min(np.linalg.eigvalsh(b).min() for b in Hmm) >= -1e-14


# ---------------------------------------------------------------- closed form (golden)
def two_plane_scene(delta, grid):
    ax = np.linspace(-0.5, 0.5, grid)
    gx, gy = np.meshgrid(ax, ax)
    gx, gy = gx.ravel(), gy.ravel()
    n = gx.shape[0]
    x = np.concatenate([gx, gx])
    y = np.concatenate([gy, gy])
    z = np.concatenate([np.zeros(n), np.full(n, delta)])
    scan = np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)])
    vox = np.zeros(2 * n, np.int32)
    poses = np.tile(np.array([1.0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]), (2, 1))
    return x, y, z, scan, vox, poses


def test_two_plane_closed_form(orc):
    with open(os.path.join(GOLDEN, "two_plane_offset.json")) as f:
        gold = json.load(f)
    x, y, z, scan, vox, poses = two_plane_scene(gold["delta"], gold["grid"])
    cl = orc.points_to_clusters(x, y, z, scan, vox, 1, 2)
    e = gold["expected"]
    c, g, Hmm, _ = orc.evaluate(orc.MM, cl, poses)
    _, _, Hc, _ = orc.evaluate(orc.COUPLED, cl, poses)
    _, _, He, _ = orc.evaluate(orc.EXACT, cl, poses)
    tz0, tz1 = 5, 11
    assert abs(c - e["cost"]) <= 1e-15
    assert abs(g[tz0] - e["grad_tz0"]) <= 1e-14 and abs(g[tz1] - e["grad_tz1"]) <= 1e-14
    assert abs(Hmm[1, 5, 5] - e["H_MM_tz1_tz1"]) <= 1e-14
    assert abs(Hc[tz1, tz1] - e["H_C_tz1_tz1"]) <= 1e-14
    assert abs(He[tz1, tz1] - e["H_E_tz1_tz1"]) <= 1e-12
    assert abs(Hc[tz0, tz1] - e["H_C_tz0_tz1"]) <= 1e-14
    assert abs(He[tz0, tz1] - e["H_E_tz0_tz1"]) <= 1e-12


# ---------------------------------------------------------------- P12: solves
def test_solve_against_lapack(orc, tiny):
    sc, cl = tiny
    T = sc.poses_init
    mu = 0.37
    _, g, Hmm, _ = orc.evaluate(orc.MM, cl, T)
    dx, info = orc.solve(orc.MM, sc.n_scans, Hmm, g, mu)
    assert info == 0
    fl = 1e-12 * max(np.diag(b).max() for b in Hmm)
    for j in range(sc.n_scans):
        A = Hmm[j] + mu * np.diag(np.maximum(np.diag(Hmm[j]), fl))
        ref = np.linalg.solve(A, -g[6 * j:6 * j + 6])
        assert np.abs(dx[6 * j:6 * j + 6] - ref).max() <= 1e-12 * np.abs(ref).max()
    _, _, Hc, _ = orc.evaluate(orc.COUPLED, cl, T)
    dx, info = orc.solve(orc.COUPLED, sc.n_scans, Hc, g, mu)
    assert info == 0
    A = Hc + mu * np.diag(np.maximum(np.diag(Hc), 1e-12 * np.diag(Hc).max()))
    ref = np.linalg.solve(A, -g)
    assert np.linalg.norm(dx - ref) <= 1e-10 * np.linalg.norm(ref)


def test_solve_reports_failed_pivot(orc):
    H = np.diag([1.0, 2.0, -3.0, 4.0, 5.0, 6.0])[None]
    g = np.ones(6)
    dx, info = orc.solve(orc.MM, 1, H, g, 0.0)
    assert info == 3 and np.all(dx == 0)
    Hd = np.diag(np.r_[np.ones(6), np.array([1.0, -1, 1, 1, 1, 1])])
    dx, info = orc.solve(orc.COUPLED, 2, Hd, np.ones(12), 0.0)
    assert info == 8 and np.all(dx == 0)


# ---------------------------------------------------------------- P13, P14: LM end to end
def align_to_pose0(P, T):
    """Apply the one global rigid motion that maps estimated pose 0 onto true
    pose 0 (the cost is invariant under it: the gauge), return aligned poses."""
    Re0, Rt0 = P[0, :9].reshape(3, 3), T[0, :9].reshape(3, 3)
    G = Rt0 @ Re0.T
    gt = T[0, 9:] - G @ P[0, 9:]
    return scenes.rigid_transform_poses(P, G, gt)


def test_lm_noise_free_recovers_truth(orc):
    sc = scenes.tiny_config(seed=1003, sigma=0.0)
    cl = orc.scene_clusters(sc)
    P, rep, cf = orc.lm(orc.MM, cl, sc.poses_init, 40)
    assert cf <= 1e-14
    A = align_to_pose0(P, sc.poses_true)
    assert np.abs(A[:, 9:] - sc.poses_true[:, 9:]).max() <= 1e-6
    rot_err = [np.linalg.norm(Rotation.from_matrix(A[j, :9].reshape(3, 3) @ sc.poses_true[j, :9].reshape(3, 3).T)
                              .as_rotvec()) for j in range(sc.n_scans)]
    assert max(rot_err) <= 1e-7


def test_lm_modes_reach_same_minimum(orc, tiny):
    sc, cl = tiny
    _, rep_m, cm = orc.lm(orc.MM, cl, sc.poses_init, 40)
    _, rep_c, cc = orc.lm(orc.COUPLED, cl, sc.poses_init, 40)
    assert abs(cm - cc) <= 1e-9 * cm
    for rep in (rep_m, rep_c):
        acc = rep[:, 4] > 0
        costs = np.r_[rep[0, 0], rep[acc, 1]]
        assert np.all(np.diff(costs) <= 1e-15)


def test_lm_stops_after_consecutive_rejections(orc):
    """The stagnation stop: after max_rejects rejected steps in a row the loop
    ends (near the optimum no step can be confirmed against the cost's
    rounding); without it the loop runs to max_iters."""
    import scenes
    sc = scenes.tiny_config(seed=1000)
    cl = orc.scene_clusters(sc)
    _, rep_full, _ = orc.lm(orc.MM, cl, sc.poses_init, 60)
    assert rep_full.shape[0] == 60
    P, rep, c = orc.lm(orc.MM, cl, sc.poses_init, 60, max_rejects=4)
    k = rep.shape[0]
    assert k < 60
    assert np.all(rep[-4:, 4] == 0)
    assert np.array_equal(rep, rep_full[:k])
    # no earlier run of 4 rejections
    acc = rep[:, 4]
    for i in range(k - 4):
        assert np.any(acc[i:i + 4] == 1)


def test_hybrid_exact_newton_converges_superlinearly(orc):
    """Coupled LM switching to the exact Hessian below a gradient norm of 0.1:
    identical to plain coupled LM before the switch, then the local Newton
    steps of the exact Hessian converge superlinearly, reaching ||g|| < 1e-8
    in fewer iterations than the linearly converging coupled steps."""
    sc = scenes.scaled_window(seed=2004, n_scans=30, n_planes=1500)
    cl = orc.scene_clusters(sc)
    _, rc, _ = orc.lm(orc.COUPLED, cl, sc.poses_init, 25, tol_g=0.0)
    _, rh, _ = orc.lm(orc.COUPLED, cl, sc.poses_init, 25, tol_g=0.0, exact_below=0.1)
    first = int(np.argmax(rc[:, 5] < 0.1))          # first evaluation below the switch
    assert first >= 1
    # the steps before the switch are the coupled ones; the switch step starts
    # from the same cost
    assert np.array_equal(rc[:first, :5], rh[:first, :5]) and rc[first, 0] == rh[first, 0]
    reach = lambda r: int(np.argmax(r[:, 5] < 1e-8)) if np.any(r[:, 5] < 1e-8) else 99
    assert reach(rh) < reach(rc)
    # quadratic phase: after the switch each accepted step at least squares
    # the gradient norm's ratio to the switch value
    g = rh[first:, 5]
    acc = rh[first:, 4] > 0
    k = np.flatnonzero(acc)[:2]
    assert g[k[0] + 1] <= 0.1 * g[k[0]]


def test_eval_abs_scales_bound_and_match(orc):
    """The per-entry absolute scales of evaluate_abs leave the outputs of
    evaluate unchanged, bound them elementwise, and equal them where each
    entry has a single contribution (one voxel, each pose one cluster)."""
    import scenes
    sc = scenes.tiny_config(seed=1000)
    cl = orc.scene_clusters(sc)
    for mode in (orc.MM, orc.COUPLED):
        c, g, H, _ = orc.evaluate(mode, cl, sc.poses_init)
        c2, g2, H2, ga, Ha = orc.evaluate_abs(mode, cl, sc.poses_init)
        assert c == c2 and np.array_equal(g, g2) and np.array_equal(H, H2)
        assert np.all(ga >= np.abs(g)) and np.all(Ha >= np.abs(H))
    one = scenes.small_scene(seed=81, n_scans=3, n_planes=1, m_range=(3, 3), pts_per_obs=(20, 20))
    cl1 = orc.scene_clusters(one)
    _, g, H, ga, Ha = orc.evaluate_abs(orc.MM, cl1, one.poses_init)
    assert np.array_equal(ga, np.abs(g)) and np.array_equal(Ha, np.abs(H))
