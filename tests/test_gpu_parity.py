"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Tolerances (all-FP64 path): relative 1e-12 for the cost, gradient (against
||g_ref||, or 1e-3 of the summed absolute contributions when ||g_ref|| is
smaller) and Hessian (Frobenius); clusters to a few ulp; LM traces must take
the same accept/reject decisions.
"""
import sys

import numpy as np
import pytest

import scenes
from helpers import block_err_g, block_err_h, build_gpu, cost_floor, grad_rel_err, rel, resolved_prefix

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


@pytest.fixture(scope="module")
def ba():
    import os
    from paper_2608_14266_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2608_14266_amd as m
    m.load()
    return m


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def mm_dense(H):
    n = H.shape[0]
    D = np.zeros((6 * n, 6 * n))
    for j in range(n):
        D[6 * j:6 * j + 6, 6 * j:6 * j + 6] = H[j]
    return D


def g_abs_scale(orc, cl, poses, sc=None):
    # the problem's gradient scale: the norm of the oracle gradient at the
    # perturbed start (a gradient that is zero in exact arithmetic, e.g. at
    # the noise-free truth, is compared against 1e-12 of it)
    start = sc.poses_init if sc is not None else poses
    _, g, _, _ = orc.evaluate(orc.MM, cl, start)
    return 1e3 * np.linalg.norm(g)


SCENES = {
    "tiny": lambda: scenes.tiny_config(seed=1000, shuffle=True),
    "tiny-noisefree": lambda: scenes.tiny_config(seed=1001, sigma=0.0),
    "window-60": lambda: scenes.scaled_window(seed=2001, n_scans=60, n_planes=3000),
}


@pytest.fixture(scope="module", params=list(SCENES))
def case(request, orc):
    sc = SCENES[request.param]()
    return request.param, sc, orc.scene_clusters(sc)


# ---------------------------------------------------------------- a0: clusters
def test_build_clusters_match_oracle(ba, dev, orc, case):
    name, sc, cl = case
    say(f"build_clusters {name}")
    prob = build_gpu(ba, sc, dev)
    info = prob.info()
    assert info["n_clusters"] == cl.C and info["n_scans"] == sc.n_scans
    vox, scan, cnt, mu, S = [t.cpu().numpy() for t in prob.export_clusters()]
    assert np.array_equal(vox, cl.vox) and np.array_equal(scan, cl.scan)
    assert np.array_equal(cnt, cl.n.astype(np.float64))
    assert np.all(np.abs(mu - cl.mu) <= 4e-16 * np.maximum(np.abs(cl.mu), 1.0))
    sc_ = np.abs(cl.S).max(axis=1, keepdims=True)
    assert np.all(np.abs(S - cl.S) <= 1e-13 * sc_)


def test_build_from_sums_match_oracle(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"build_clusters_from_sums {name}")
    v, s, n, s1, s2 = orc.points_to_raw_sums(sc.x, sc.y, sc.z, sc.scan, sc.voxel)
    mu_ref, S_ref = orc.center_raw_sums(n, s1, s2)
    rng = np.random.default_rng(4)
    perm = rng.permutation(v.shape[0])   # any input order
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a[perm]), dtype=dt, device=dev)
    prob = ba.build_clusters_from_sums(t(v, torch.int32), t(s, torch.int32), t(n, torch.int64),
                                       t(s1, torch.float64), t(s2, torch.float64), sc.n_scans, sc.n_voxels)
    vox, scan, cnt, mu, S = [x.cpu().numpy() for x in prob.export_clusters()]
    assert np.array_equal(vox, v) and np.array_equal(scan, s)
    assert np.all(np.abs(mu - mu_ref) <= 2.3e-16 * np.maximum(np.abs(mu_ref), 1e-300))
    assert np.all(np.abs(S - S_ref) <= 2.3e-16 * np.abs(S_ref) + 1e-300)


# ---------------------------------------------------------------- a1-a4: evaluation
@pytest.mark.parametrize("chunk_len", [0, 64])
def test_eval_mm_matches_oracle(ba, dev, orc, case, chunk_len):
    import torch
    name, sc, cl = case
    say(f"eval MM {name} chunk_len={chunk_len}")
    prob = build_gpu(ba, sc, dev, chunk_len=chunk_len)
    for poses in (sc.poses_init, sc.poses_true):
        P = torch.as_tensor(poses, device=dev)
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
        c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, poses)
        c = cost.cpu().numpy()[0]
        assert abs(c - c_ref) <= TOL * abs(c_ref) + cost_floor(orc, cl, poses)
        G = g_abs_scale(orc, cl, poses, sc)
        assert grad_rel_err(g.cpu().numpy().ravel(), g_ref, G) <= TOL
        assert rel(H.cpu().numpy(), H_ref) <= TOL
        # per pose block, each against its own rounding scale, floored at the
        # block's scale at the perturbed start (at the noise-free truth every
        # gradient term vanishes in exact arithmetic: both sides' terms are
        # rounding noise there, as in the global floor)
        _, _, _, ga0, Ha0 = orc.evaluate_abs(orc.MM, cl, sc.poses_init)
        eg = block_err_g(g.cpu().numpy(), g_ref, np.maximum(ga, ga0))
        eh = block_err_h(H.cpu().numpy(), H_ref, np.maximum(Ha, Ha0))
        print(f"  {name}: worst gradient block {eg:.2e}, Hessian block {eh:.2e}")
        assert eg <= TOL and eh <= TOL


def test_cost_only_matches(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"cost only {name}")
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM, derivatives=False)
    assert g is None and H is None
    c_ref = orc.cost(cl, sc.poses_init)
    assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref


def test_voxel_eigen_matches(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"voxel eig {name}")
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev)
    _, _, _, eig = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM, derivatives=False, voxel_eig=True)
    eig = eig.cpu().numpy()
    st = orc.voxel_stats(cl, sc.poses_init)
    lam, U = st["lam"], st["U"]
    seen = np.isin(np.arange(sc.n_voxels), cl.vox)
    assert np.all(np.isnan(eig[~seen, 0]))
    e = eig[seen]
    # per-voxel lambda_min: any backward-stable eigen-solver leaves an absolute
    # error of a few eps ||A|| = eps lambda_2, and forming A from up to 100
    # clusters at world coordinates of ~100 m adds the rounding of the centroid
    # offsets, relative to lambda_0 (reading of the tolerance: see the design
    # notes, per-voxel eigenvalue bound)
    err = np.abs(e[:, 0] - lam[seen, 0])
    bound = 1e-12 * lam[seen, 0] + 1e-13 * lam[seen, 2]
    print("worst lambda_min error / bound", float(np.max(err / bound)))
    assert np.all(err <= bound)
    dots = np.abs(np.einsum("vi,vi->v", e[:, 1:], U[seen][:, :, 0]))
    assert np.all(dots >= 1 - 1e-12)


# ---------------------------------------------------------------- a5: solve
def test_solve_mm_matches_oracle(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"solve MM {name}")
    _, g, H, _ = orc.evaluate(orc.MM, cl, sc.poses_init)
    for mu in (0.0, 1e-2, 3.7):
        dx, info = ba.solve_increment(ba.MODE_MM, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), mu)
        ref, info_ref = orc.solve(orc.MM, sc.n_scans, H, g, mu)
        # the exact surrogate Hessian can be indefinite away from the optimum:
        # undamped, both sides must report the same failing pivot
        assert int(info.cpu().numpy()[0]) == info_ref
        if mu > 0:
            assert info_ref == 0
        assert rel(dx.cpu().numpy().ravel(), ref) <= TOL


def test_solve_mm_reports_pivot(ba, dev, orc):
    import torch
    say("solve MM failing pivot")
    H = np.tile(np.eye(6), (3, 1, 1))
    H[1, 2, 2] = -1.0
    g = np.ones(18)
    dx, info = ba.solve_increment(ba.MODE_MM, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), 0.0)
    ref, info_ref = orc.solve(orc.MM, 3, H, g, 0.0)
    assert int(info.cpu().numpy()[0]) == info_ref == 9
    assert np.all(dx.cpu().numpy() == 0)


# ---------------------------------------------------------------- a6: LM iterations
@pytest.mark.parametrize("iters", [10, 20])
def test_iterate_mm_matches_oracle(ba, dev, orc, case, iters):
    import torch
    name, sc, cl = case
    say(f"iterate MM {name} iters={iters}")
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(prob, P, ba.MODE_MM, max_iters=iters)
    P_ref, rep_ref, c_ref = orc.lm(orc.MM, cl, sc.poses_init, iters)
    tr = tr[:, 0, :]
    assert tr.shape[0] == rep_ref.shape[0] == iters
    k = resolved_prefix(tr, rep_ref)
    assert k >= min(iters, 8)
    # while decisions are resolved, the traces agree step by step
    assert np.array_equal(tr[:k, 4], rep_ref[:k, 4])
    scale = np.maximum(np.abs(rep_ref[:k, [0, 1]]), 1e-3 * rep_ref[0, 0])
    assert np.all(np.abs(tr[:k, [0, 1]] - rep_ref[:k, [0, 1]]) <= TOL * scale)
    assert np.all(np.abs(tr[:k, 3] - rep_ref[:k, 3]) <= 1e-9 * rep_ref[:k, 3])
    # end state: the same minimum
    assert abs(reps[0]["cost_final"] - c_ref) <= TOL * max(c_ref, 1e-3 * rep_ref[0, 0])
    dP = np.abs(P.cpu().numpy() - P_ref)
    if k == iters:
        ptol = 1e-11
    else:
        # past the resolved prefix each side may accept or reject steps whose
        # cost change is below the resolution c_res = 1e-11 c + 1e-12 c0, i.e.
        # moves of up to sqrt(2 c_res / h_min) along the flattest direction
        _, _, H_end, _ = orc.evaluate(orc.MM, cl, P_ref)
        h_min = min(np.linalg.eigvalsh(Hj)[0] for Hj in H_end if np.any(Hj))
        c_res = 1e-11 * c_ref + 1e-12 * rep_ref[0, 0]
        ptol = 3.0 * np.sqrt(2.0 * c_res / h_min)
        print(f"unresolved tail from iteration {k}: pose tolerance {ptol:.2e}, max difference {dP.max():.2e}")
    assert np.all(dP <= ptol * (1.0 + np.abs(P_ref)))


# ---------------------------------------------------------------- edge cases
def test_edge_unobserved_scan_and_voxel_gaps(ba, dev, orc):
    import torch
    say("edge: unobserved scan, voxel id gaps, single-scan voxels")
    sc = scenes.small_scene(seed=77, n_scans=6, n_planes=40, m_range=(1, 3), pts_per_obs=(5, 30),
                            path_len=8.0, offset_range=8.0)
    keep = sc.scan != 3                       # scan 3 observes nothing
    for k in ("x", "y", "z", "scan", "voxel"):
        setattr(sc, k, getattr(sc, k)[keep])
    sc.voxel = (sc.voxel * 3 + 1).astype(np.int32)   # ids with gaps
    sc.n_voxels = 3 * 40 + 2
    cl = orc.scene_clusters(sc)
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sc.poses_init)
    assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref
    gg = g.cpu().numpy()
    assert np.all(gg[3] == 0) and np.all(H.cpu().numpy()[3] == 0)
    assert grad_rel_err(gg.ravel(), g_ref, g_abs_scale(orc, cl, sc.poses_init)) <= TOL
    assert rel(H.cpu().numpy(), H_ref) <= TOL
    assert block_err_g(gg, g_ref, ga) <= TOL and block_err_h(H.cpu().numpy(), H_ref, Ha) <= TOL
    P2 = P.clone().contiguous()
    reps, tr = ba.iterate(prob, P2, ba.MODE_MM, max_iters=8)
    P_ref, rep_ref, _ = orc.lm(orc.MM, cl, sc.poses_init, 8)
    k = resolved_prefix(tr[:, 0, :], rep_ref)
    assert np.array_equal(tr[:k, 0, 4], rep_ref[:k, 4])
    assert np.array_equal(P2.cpu().numpy()[3], sc.poses_init[3])
    assert np.all(np.abs(P2.cpu().numpy() - P_ref) <= 1e-11 * (1 + np.abs(P_ref)))


def test_edge_voxel_seen_by_more_than_a_wave(ba, dev, orc):
    import torch
    say("edge: voxels observed by 100 scans")
    sc = scenes.small_scene(seed=78, n_scans=100, n_planes=5, m_range=(70, 100), pts_per_obs=(4, 9),
                            path_len=30.0, offset_range=20.0)
    cl = orc.scene_clusters(sc)
    prob = build_gpu(ba, sc, dev, chunk_len=64)
    assert prob.info()["max_m"] >= 70
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sc.poses_init)
    assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref
    assert grad_rel_err(g.cpu().numpy().ravel(), g_ref, g_abs_scale(orc, cl, sc.poses_init)) <= TOL
    assert rel(H.cpu().numpy(), H_ref) <= TOL
    assert block_err_g(g.cpu().numpy(), g_ref, ga) <= TOL and block_err_h(H.cpu().numpy(), H_ref, Ha) <= TOL


def test_edge_single_cluster(ba, dev, orc):
    import torch
    say("edge: one cluster")
    sc = scenes.small_scene(seed=79, n_scans=1, n_planes=1, m_range=(1, 1), pts_per_obs=(3, 3))
    cl = orc.scene_clusters(sc)
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    c_ref, g_ref, H_ref, _ = orc.evaluate(orc.MM, cl, sc.poses_init)
    assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref + cost_floor(orc, cl, sc.poses_init)
    # a one-cluster voxel has zero gradient in exact arithmetic: rounding only
    hn = np.abs(H_ref).max()
    assert np.abs(g.cpu().numpy()).max() <= 1e-12 * max(1.0, hn)
    assert np.abs(g_ref).max() <= 1e-12 * max(1.0, hn)
    assert rel(H.cpu().numpy(), H_ref) <= TOL


def test_invalid_inputs_rejected(ba, dev):
    import torch
    say("edge: invalid labels and coordinates")
    sc = scenes.tiny_config(seed=1000)
    x, y, z, s, v = [t.clone() for t in __import__("helpers").to_dev(sc, dev)]
    s[5] = sc.n_scans
    with pytest.raises(ba.BAError) as ei:
        ba.build_clusters(x, y, z, s, v, sc.n_scans, sc.n_voxels)
    assert ei.value.status == -1
    x, y, z, s, v = [t.clone() for t in __import__("helpers").to_dev(sc, dev)]
    x[7] = float("nan")
    with pytest.raises(ba.BAError):
        ba.build_clusters(x, y, z, s, v, sc.n_scans, sc.n_voxels)


def test_deterministic_bitwise(ba, dev, orc):
    import torch
    say("determinism: two builds, two evaluations")
    sc = scenes.scaled_window(seed=2002, n_scans=40, n_planes=2000)
    outs = []
    for rep in range(2):
        prob = build_gpu(ba, sc, dev)
        P = torch.as_tensor(sc.poses_init, device=dev)
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
        P2 = P.clone().contiguous()
        ba.iterate(prob, P2, ba.MODE_MM, max_iters=5)
        outs.append([t.cpu().numpy().copy() for t in (cost, g, H, P2)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_iterate_stops_after_consecutive_rejections(ba, dev, orc):
    import torch
    say("LM stagnation stop")
    sc = scenes.tiny_config(seed=1000)
    cl = orc.scene_clusters(sc)
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(prob, P, ba.MODE_MM, max_iters=60, max_rejects=4)
    r = reps[0]
    assert r["stalled"] == 1 and r["converged"] == 0 and r["iters"] < 60
    tr = tr[: r["iters"], 0, :]
    assert np.all(tr[-4:, 4] == 0)
    _, rep_ref, c_ref = orc.lm(orc.MM, cl, sc.poses_init, 60, max_rejects=4)
    assert abs(r["cost_final"] - c_ref) <= 1e-12 * c_ref
