"""Parity of the bottom-up multi-level voxelization and planarity selection
(Sec. IV-A, Eq. 4-5, Alg. 1) with the oracle: per-level cluster and cell
counts exactly, the kept cells, their clusters (scan and count exactly, sums
to rounding), the problem built from them, determinism and input errors.

Planarity decisions whose ratio lies within rounding of tau may go either
way; the comparison skips those cells (both outcomes are correct)."""
import numpy as np
import pytest

import scenes
from helpers import build_gpu_sums, cost_floor, grad_rel_err, rel
from oracle import voxelize as ovx

pytestmark = pytest.mark.gpu

BORDER = 1e-9        # |l0 - tau l1| below this fraction of l2 counts as undecided
RANK_BORDER = 1e-12  # |l1 - 1e-10 l2| below this fraction of l2 counts as undecided


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
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


def _dev(a, dt, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def _run(ba, dev, x, y, z, scan, poses, d, L, tau, min_scans=1):
    import torch
    m = ba.voxelize(_dev(x, torch.float64, dev), _dev(y, torch.float64, dev), _dev(z, torch.float64, dev),
                    _dev(scan, torch.int32, dev), _dev(poses, torch.float64, dev), d, L, tau, min_scans)
    try:
        inf = m.info()
        out = {k: v.cpu().numpy() for k, v in m.export().items()}
    finally:
        m.close()
    return inf, out


def _compare(inf, out, ref, tau):
    lv = ref["levels"]
    assert inf["level_clusters"] == [l["cell"].shape[0] for l in lv]
    assert inf["level_voxels"] == [l["n_voxels"] for l in lv]
    # kept cells: (level, cell) in output order on both sides, undecided ones aside
    und = set()
    ref_keep = []
    for k, l in enumerate(lv):
        lam = l["lam"]
        # undecided: the rank test within rounding of its threshold, or the
        # ratio test within rounding where the rank test clearly passes
        rank_gap = lam[:, 1] - ovx.RANK2 * lam[:, 2]
        rank_border = np.abs(rank_gap) <= RANK_BORDER * lam[:, 2]
        ratio_border = np.abs(lam[:, 0] - tau * lam[:, 1]) <= BORDER * lam[:, 2]
        border = (rank_border | ((rank_gap > 0) & ratio_border)) & (l["n_points"] >= 3)
        cells = l["cell"][l["vstart"]]
        for v in range(l["n_voxels"]):
            key = (k + 1,) + tuple(int(c) for c in cells[v])
            if border[v]:
                und.add(key)
            elif l["keep"][v]:
                ref_keep.append(key)
    got = [(int(a),) + tuple(int(c) for c in b) for a, b in zip(out["voxel_level"], out["voxel_cell"])]
    assert [g for g in got if g not in und] == ref_keep
    # clusters of every cell kept on both sides
    ro = ref["out"]
    rkeys = [(int(a),) + tuple(int(c) for c in b) for a, b in zip(ro["voxel_level"], ro["voxel_cell"])]
    rpos = {k: i for i, k in enumerate(rkeys)}
    for gv, key in enumerate(got):
        if key not in rpos:
            continue
        rv = rpos[key]
        gsel = out["voxel"] == gv
        rsel = ro["voxel"] == rv
        assert np.array_equal(out["scan"][gsel], ro["scan"][rsel])
        assert np.array_equal(out["count"][gsel], ro["count"][rsel])
        assert np.allclose(out["sum"][gsel], ro["sum"][rsel], rtol=1e-12, atol=1e-12)
        assert np.allclose(out["sumsq"][gsel], ro["sumsq"][rsel], rtol=1e-12, atol=1e-10)
    return len(und)


def _cloud(seed, n, n_scans, spread=4.0):
    rng = np.random.default_rng(seed)
    x, y, z = rng.uniform(-spread, spread, (3, n))
    scan = rng.integers(0, n_scans, n).astype(np.int32)
    P = np.zeros((n_scans, 12))
    for j in range(n_scans):
        a = rng.uniform(-np.pi, np.pi)
        c, s = np.cos(a), np.sin(a)
        P[j, :9] = [c, -s, 0, s, c, 0, 0, 0, 1]
        P[j, 9:] = rng.uniform(-5, 5, 3)
    return x, y, z, scan, P


@pytest.mark.parametrize("seed,n,n_scans,d,L,tau,min_scans", [
    (1, 3000, 4, 0.7, 3, 0.5, 1),     # isotropic noise: many cells either way
    (2, 20000, 9, 0.31, 4, 0.2, 2),   # several levels, min_scans
    (3, 1, 1, 1.0, 2, 0.5, 1),        # one point: no planar cell
    (4, 500, 1, 2.0, 1, 0.9, 1),      # one scan (no scan bits), one level
])
def test_voxelize_random_clouds_match_oracle(ba, dev, seed, n, n_scans, d, L, tau, min_scans):
    say(f"voxelize random cloud seed {seed} n {n}")
    x, y, z, scan, P = _cloud(seed, n, n_scans)
    inf, out = _run(ba, dev, x, y, z, scan, P, d, L, tau, min_scans)
    ref = ovx.voxelize(x, y, z, scan, P, d, L, tau, min_scans)
    nund = _compare(inf, out, ref, tau)
    assert nund <= 2


@pytest.mark.parametrize("tau,min_scans", [(0.05, 2), (0.01, 1)])
def test_voxelize_window_scene_matches_oracle(ba, dev, tau, min_scans):
    """Planar patches of the window law (60 scans, 3000 planes, 1 m patches,
    3 cm noise) at the perturbed initial poses, three levels from d = 0.5 m."""
    sc = scenes.scaled_window(seed=2001, n_scans=60, n_planes=3000)
    say(f"voxelize window scene: {sc.n_points} points, tau {tau}")
    inf, out = _run(ba, dev, sc.x, sc.y, sc.z, sc.scan, sc.poses_init, 0.5, 3, tau, min_scans)
    ref = ovx.voxelize(sc.x, sc.y, sc.z, sc.scan, sc.poses_init, 0.5, 3, tau, min_scans)
    _compare(inf, out, ref, tau)
    assert inf["n_voxels"] > 1000


def test_voxelize_then_build_matches_oracle_problem(ba, dev, orc):
    """The kept clusters equal the oracle's voxelization (ids, scans and
    counts exactly, sums to rounding) and build a problem whose residual,
    gradient and Hessian equal the oracle's on the same clusters."""
    import torch
    sc = scenes.scaled_window(seed=2003, n_scans=40, n_planes=2000)
    x, y, z, s, P0 = sc.x, sc.y, sc.z, sc.scan, sc.poses_init
    inf, out = _run(ba, dev, x, y, z, s, P0, 0.5, 2, 0.05, 2)
    ro = ovx.voxelize(x, y, z, s, P0, 0.5, 2, 0.05, 2)["out"]
    assert np.array_equal(out["voxel"], ro["voxel"]) and np.array_equal(out["scan"], ro["scan"])
    assert np.array_equal(out["count"], ro["count"])
    assert np.allclose(out["sum"], ro["sum"], rtol=1e-12, atol=1e-12)
    assert np.allclose(out["sumsq"], ro["sumsq"], rtol=1e-12, atol=1e-10)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    prob = ba.build_clusters_from_sums(t(out["voxel"], torch.int32), t(out["scan"], torch.int32),
                                       t(out["count"], torch.int64), t(out["sum"], torch.float64),
                                       t(out["sumsq"], torch.float64), sc.n_scans, inf["n_voxels"])
    try:
        P = t(sc.poses_init, torch.float64)
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    finally:
        prob.close()
    # the oracle on the same clusters (its own centring of the raw sums)
    order = np.lexsort((out["scan"], out["voxel"]))
    mu, S = orc.center_raw_sums(out["count"][order], out["sum"][order], out["sumsq"][order])
    cl = orc.Clusters(out["voxel"][order].astype(np.int32), out["scan"][order].astype(np.int32),
                      out["count"][order].astype(np.int64), mu, S, inf["n_voxels"], sc.n_scans)
    c_ref, g_ref, H_ref, _ = orc.evaluate(orc.MM, cl, sc.poses_init)
    assert abs(float(cost.cpu()[0]) - c_ref) <= 1e-12 * c_ref + cost_floor(orc, cl, sc.poses_init)
    assert grad_rel_err(g.cpu().numpy().ravel(), g_ref, np.abs(g_ref).sum()) <= 1e-12
    assert rel(H.cpu().numpy(), H_ref) <= 1e-12


def test_voxelize_is_deterministic(ba, dev):
    x, y, z, scan, P = _cloud(7, 50000, 6)
    a = _run(ba, dev, x, y, z, scan, P, 0.4, 3, 0.3)[1]
    b = _run(ba, dev, x, y, z, scan, P, 0.4, 3, 0.3)[1]
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_voxelize_rejects_bad_input(ba, dev):
    x, y, z, scan, P = _cloud(8, 100, 3)
    bad_scan = scan.copy()
    bad_scan[5] = 3
    with pytest.raises(ba.BAError, match="scan out of range"):
        _run(ba, dev, x, y, z, bad_scan, P, 0.5, 2, 0.3)
    xn = x.copy()
    xn[7] = np.nan
    with pytest.raises(ba.BAError, match="non-finite"):
        _run(ba, dev, xn, y, z, scan, P, 0.5, 2, 0.3)
    with pytest.raises(ba.BAError, match="beyond 2\\^30"):
        _run(ba, dev, x * 1e6, y, z, scan, P, 1e-4, 2, 0.3)
    with pytest.raises(ba.BAError, match="options out of range"):
        _run(ba, dev, x, y, z, scan, P, 0.0, 2, 0.3)
    with pytest.raises(ba.BAError, match="options out of range"):
        _run(ba, dev, x, y, z, scan, P, 0.5, 17, 0.3)


# ---------------------------------------------------------------- host stream (adaptive loader)
def _run_host(ba, dev, x, y, z, scan, poses, d, L, tau, min_scans=1, **so):
    import torch
    m = ba.voxelize_host(x, y, z, scan, torch.as_tensor(poses, device=dev), d, L, tau, min_scans, **so)
    try:
        inf = m.info()
        out = {k: v.cpu().numpy() for k, v in m.export().items()}
    finally:
        m.close()
    return inf, out


def _same_map(a, b):
    """Equal cells, scans and counts; sums equal to rounding (the batches add
    their partial sums in another order)."""
    for k in ("voxel", "scan", "count", "voxel_level", "voxel_cell"):
        assert np.array_equal(a[k], b[k]), k
    assert np.allclose(a["sum"], b["sum"], rtol=1e-13, atol=1e-13)
    assert np.allclose(a["sumsq"], b["sumsq"], rtol=1e-13, atol=1e-11)


def test_host_stream_in_many_batches_matches_oracle_and_device_path(ba, dev):
    x, y, z, scan, P = _cloud(11, 20_000, 9)
    say("voxelize_host: 20000 points in batches of 1024")
    inf, out = _run_host(ba, dev, x, y, z, scan, P, 0.31, 4, 0.2, 2, batch_points=1024)
    assert inf["n_batches"] == 20
    ref = ovx.voxelize(x, y, z, scan, P, 0.31, 4, 0.2, 2)
    _compare(inf, out, ref, 0.2)
    _, dout = _run(ba, dev, x, y, z, scan, P, 0.31, 4, 0.2, 2)
    _same_map(out, dout)


def test_host_stream_window_scene_pinned_and_pageable(ba, dev):
    import torch
    sc = scenes.scaled_window(seed=2001, n_scans=60, n_planes=3000)
    say(f"voxelize_host: window scene {sc.n_points} points, pageable and pinned")
    _, dout = _run(ba, dev, sc.x, sc.y, sc.z, sc.scan, sc.poses_init, 0.5, 3, 0.05, 2)
    inf, out = _run_host(ba, dev, sc.x, sc.y, sc.z, sc.scan, sc.poses_init, 0.5, 3, 0.05, 2, batch_points=50_000)
    assert inf["n_batches"] == (sc.n_points + 49_999) // 50_000
    _same_map(out, dout)
    pin = lambda a, dt: torch.as_tensor(a, dtype=dt).pin_memory()
    px, py, pz = pin(sc.x, torch.float64), pin(sc.y, torch.float64), pin(sc.z, torch.float64)
    ps = pin(sc.scan, torch.int32)
    _, out2 = _run_host(ba, dev, px, py, pz, ps, sc.poses_init, 0.5, 3, 0.05, 2, batch_points=50_000)
    _same_map(out2, dout)
    inf3, out3 = _run_host(ba, dev, px, py, pz, ps, sc.poses_init, 0.5, 3, 0.05, 2)   # one batch
    assert inf3["n_batches"] == 1
    _same_map(out3, dout)


def test_host_stream_rejects_bad_options(ba, dev):
    x, y, z, scan, P = _cloud(12, 100, 2)
    with pytest.raises(ba.BAError, match="stream options out of range"):
        _run_host(ba, dev, x, y, z, scan, P, 0.5, 2, 0.3, alpha=1.5)
    with pytest.raises(ba.BAError, match="stream options out of range"):
        _run_host(ba, dev, x, y, z, scan, P, 0.5, 2, 0.3, batch_points=-1)
