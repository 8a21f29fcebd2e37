"""GPU tests of the batched form: many uneven windows in one problem, one
launch per pass for all windows, the whole LM captured in one HIP graph, and
the autotuned launch choices.

Bar: each window's result inside the batch is bitwise identical to the same
window solved as a problem of its own (per-window reductions never mix
windows); batched evaluations match the FP64 oracle per window at 1e-12;
other launch choices move results only at the rounding level (1e-12)."""
import numpy as np
import pytest

import scenes.sums as ss
from helpers import block_err_g, block_err_h, build_gpu_sums, oracle_clusters_from_sums, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12


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


@pytest.fixture(scope="module")
def batch():
    # 7 uneven windows (8..60 poses), the batched-window law at small size
    return ss.batch_windows(seed=4100, n_windows=7, poses_range=(8, 60), vox_per_pose=40,
                            vox_range=(300, 2000), workers=1)


def _prec_kw(ba, prec, sc, dev):
    import torch
    if prec == "f64":
        return {}
    return dict(precision=ba.PREC_F32, ref_poses=torch.as_tensor(sc.poses_init, device=dev))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["mm", "coupled"])
def test_batched_windows_equal_solo_bitwise(ba, dev, batch, prec, mode):
    import torch
    say(f"batched vs solo {prec} {mode}")
    m = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    iters = 12 if mode == "mm" else 6
    pb = build_gpu_sums(ba, batch, dev, **_prec_kw(ba, prec, batch, dev))
    assert pb.info()["n_windows"] == batch.n_windows
    P = torch.as_tensor(batch.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(pb, P, m, max_iters=iters)
    Pb = P.cpu().numpy()
    s0 = 0
    for w in range(batch.n_windows):
        sw = ss.window_of(batch, w)
        ps = build_gpu_sums(ba, sw, dev, **_prec_kw(ba, prec, sw, dev))
        Q = torch.as_tensor(sw.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(ps, Q, m, max_iters=iters)
        assert np.array_equal(Q.cpu().numpy(), Pb[s0:s0 + sw.n_scans]), f"window {w} poses"
        assert np.array_equal(t1[:, 0, :], tr[:, w, :]), f"window {w} trace"
        for k in ("iters", "n_accepted", "cost_final", "gnorm_final", "mu_final", "cost_initial"):
            assert r1[0][k] == reps[w][k], (w, k)
        s0 += sw.n_scans


def test_coupled_many_windows_equal_solo_bitwise(ba, dev):
    """More windows than one dataflow launch takes (128): the coupled LM of
    windows in the first and second launch equals each window alone."""
    import torch
    sc = ss.batch_windows(seed=4300, n_windows=130, poses_range=(4, 14), vox_per_pose=20, vox_range=(100, 400),
                          workers=1)
    say(f"coupled batch of {sc.n_windows} windows")
    pb = build_gpu_sums(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(pb, P, ba.MODE_COUPLED, max_iters=4)
    pb.close()
    Pb = P.cpu().numpy()
    starts = np.concatenate([[0], np.cumsum([ss.window_of(sc, w).n_scans for w in range(sc.n_windows)])])
    for w in (0, 1, 127, 128, 129):
        sw = ss.window_of(sc, w)
        ps = build_gpu_sums(ba, sw, dev)
        Q = torch.as_tensor(sw.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(ps, Q, ba.MODE_COUPLED, max_iters=4)
        ps.close()
        assert np.array_equal(Q.cpu().numpy(), Pb[starts[w]:starts[w + 1]]), f"window {w} poses"
        assert np.array_equal(t1[:, 0, :], tr[:, w, :]), f"window {w} trace"
        for k in ("iters", "n_accepted", "cost_final", "gnorm_final", "mu_final"):
            assert r1[0][k] == reps[w][k], (w, k)


def test_coupled_long_chains_equal_solo_bitwise(ba, dev):
    """Windows of 3, 5, 6, 9 and 17 block rows of 64 (n = 6 x poses) share one
    dataflow back-substitution launch, whose tasks each wait on the pairs of
    block rows below them; every window's coupled LM run equals the window
    solved alone."""
    import torch
    sizes = (30, 53, 64, 96, 181)
    sc = ss.batch_windows(seed=4400, n_windows=len(sizes), poses=list(sizes), vox_per_pose=12,
                          vox_range=(300, 3000), workers=1)
    say(f"coupled chains: windows {sizes}, {sc.n_clusters} clusters")
    pb = build_gpu_sums(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(pb, P, ba.MODE_COUPLED, max_iters=4)
    pb.close()
    Pb = P.cpu().numpy()
    s0 = 0
    for w in range(sc.n_windows):
        sw = ss.window_of(sc, w)
        ps = build_gpu_sums(ba, sw, dev)
        Q = torch.as_tensor(sw.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(ps, Q, ba.MODE_COUPLED, max_iters=4)
        ps.close()
        assert reps[w]["n_accepted"] >= 1 and reps[w]["last_info"] == 0, (w, reps[w])
        assert np.array_equal(Q.cpu().numpy(), Pb[s0:s0 + sw.n_scans]), f"window {w} poses"
        assert np.array_equal(t1[:, 0, :], tr[:, w, :]), f"window {w} trace"
        s0 += sw.n_scans


@pytest.mark.parametrize("sizes", [(8, 255, 256, 257, 513), (255, 257, 513, 1030)])
def test_solve_forms_equal_bitwise(ba, dev, sizes):
    """The MM increment solve covers a window with one block per 256 poses,
    or, once a window of the problem exceeds 1024 poses, with one statistics
    block per window plus one thread per pose over the whole grid.  A window's
    LM run must be bitwise the same whichever form and block count its problem
    takes: windows at and around the block boundaries, solved in a batch and
    alone (the second batch runs the two-launch form, its windows alone the
    block form)."""
    import torch
    sc = ss.batch_windows(seed=4200, n_windows=len(sizes), poses=list(sizes), vox_per_pose=8,
                          vox_range=(300, 8000), workers=1)
    say(f"solve forms: windows {sizes}, {sc.n_clusters} clusters")
    pb = build_gpu_sums(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(pb, P, ba.MODE_MM, max_iters=10)
    pb.close()
    Pb = P.cpu().numpy()
    s0 = 0
    for w in range(sc.n_windows):
        sw = ss.window_of(sc, w)
        ps = build_gpu_sums(ba, sw, dev)
        Q = torch.as_tensor(sw.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(ps, Q, ba.MODE_MM, max_iters=10)
        ps.close()
        assert np.array_equal(Q.cpu().numpy(), Pb[s0:s0 + sw.n_scans]), f"window {w} poses"
        assert np.array_equal(t1[:, 0, :], tr[:, w, :]), f"window {w} trace"
        assert r1[0]["n_accepted"] >= 3, f"window {w} made no progress"
        for k in ("iters", "n_accepted", "cost_final", "gnorm_final", "mu_final"):
            assert r1[0][k] == reps[w][k], (w, k)
        s0 += sw.n_scans


def test_batched_eval_matches_oracle_per_window(ba, dev, orc, batch):
    import torch
    say("batched eval vs oracle")
    pb = build_gpu_sums(ba, batch, dev)
    P = torch.as_tensor(batch.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)
    cost = cost.cpu().numpy(); g = g.cpu().numpy().reshape(-1, 6); H = H.cpu().numpy().reshape(-1, 6, 6)
    s0 = 0
    for w in range(batch.n_windows):
        sw = ss.window_of(batch, w)
        cl = oracle_clusters_from_sums(orc, sw)
        c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sw.poses_init)
        n = sw.n_scans
        assert abs(cost[w] - c_ref) <= TOL * c_ref
        # per pose block, each against its own rounding scale
        assert block_err_g(g[s0:s0 + n], g_ref, ga) <= TOL
        assert block_err_h(H[s0:s0 + n], H_ref, Ha) <= TOL
        assert rel(H[s0:s0 + n], H_ref) <= TOL
        s0 += n


TUNINGS = [
    dict(vox_split=1, vox_grid=0, pose_grid=0, chunk_len=256),
    dict(vox_split=2, vox_grid=2, pose_grid=4, chunk_len=64),
    dict(vox_split=4, vox_grid=1, pose_grid=1, chunk_len=1024),
    dict(vox_split=4, vox_grid=8, pose_grid=8, chunk_len=32),
    dict(vox_split=0, vox_grid=0, pose_grid=0, chunk_len=512),   # split chosen per group
    dict(vox_split=0, vox_grid=2, pose_grid=2, chunk_len=128),
]


@pytest.mark.parametrize("tune", TUNINGS, ids=lambda t: "s{vox_split}g{vox_grid}p{pose_grid}c{chunk_len}".format(**t))
def test_launch_choices_keep_results(ba, dev, orc, batch, tune):
    import torch
    say(f"tuning {tune}")
    pb = build_gpu_sums(ba, batch, dev)
    P = torch.as_tensor(batch.poses_init, device=dev)
    ref = [t.cpu().numpy() for t in ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)[:3]]
    ba.problem_set_tuning(pb, tune)
    assert ba.problem_get_tuning(pb) == tune
    a = [t.cpu().numpy() for t in ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)[:3]]
    b = [t.cpu().numpy() for t in ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)[:3]]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)                  # reproducible for one setting
    assert np.all(np.abs(a[0] - ref[0]) <= TOL * np.abs(ref[0]))
    # per pose block, against the oracle's rounding scale of each block
    ga = np.concatenate([orc.evaluate_abs(orc.MM, oracle_clusters_from_sums(orc, ss.window_of(batch, w)),
                                          ss.window_of(batch, w).poses_init)[3] for w in range(batch.n_windows)])
    Ha = np.concatenate([orc.evaluate_abs(orc.MM, oracle_clusters_from_sums(orc, ss.window_of(batch, w)),
                                          ss.window_of(batch, w).poses_init)[4] for w in range(batch.n_windows)])
    assert block_err_g(a[1], ref[1], ga) <= TOL and block_err_h(a[2], ref[2], Ha) <= TOL
    assert rel(a[2], ref[2]) <= TOL
    # a captured LM run after the change replays the new launches: equal to eager
    import os
    P1 = torch.as_tensor(batch.poses_init, device=dev).contiguous()
    r1, t1 = ba.iterate(pb, P1, ba.MODE_MM, max_iters=6)
    r1b, t1b = ba.iterate(pb, P1.copy_(torch.as_tensor(batch.poses_init, device=dev)), ba.MODE_MM, max_iters=6)
    os.environ["BA_NO_GRAPH"] = "1"
    try:
        P2 = torch.as_tensor(batch.poses_init, device=dev).contiguous()
        r2, t2 = ba.iterate(pb, P2, ba.MODE_MM, max_iters=6)
    finally:
        del os.environ["BA_NO_GRAPH"]
    assert np.array_equal(t1, t2) and np.array_equal(t1b, t2)
    assert np.array_equal(P1.cpu().numpy(), P2.cpu().numpy())


def test_autotune_applies_a_valid_choice(ba, dev, batch, tmp_path):
    import torch
    say("autotune")
    pb = build_gpu_sums(ba, batch, dev)
    P = torch.as_tensor(batch.poses_init, device=dev)
    ref = [t.cpu().numpy() for t in ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)[:3]]
    cache = str(tmp_path / "tuning.json")
    t1 = ba.tuned(pb, P, cache_path=cache, reps=2)
    assert not t1["cached"] and t1["vox_split"] in (0, 1, 2, 4) and t1["chunk_len"] >= 32
    assert ba.problem_get_tuning(pb) == {k: t1[k] for k in ("vox_split", "vox_grid", "pose_grid", "chunk_len")}
    a = [t.cpu().numpy() for t in ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)[:3]]
    assert np.all(np.abs(a[0] - ref[0]) <= TOL * np.abs(ref[0])) and rel(a[2], ref[2]) <= TOL
    # a second problem of the same class takes the cached choice
    pb2 = build_gpu_sums(ba, batch, dev)
    t2 = ba.tuned(pb2, P, cache_path=cache)
    assert t2["cached"] and t2["key"] == t1["key"]
    assert ba.problem_get_tuning(pb2) == ba.problem_get_tuning(pb)


def test_bad_tuning_is_rejected(ba, dev, batch):
    pb = build_gpu_sums(ba, batch, dev)
    for bad in (dict(vox_split=3), dict(vox_grid=-1), dict(pose_grid=65), dict(chunk_len=16), dict(chunk_len=2048)):
        with pytest.raises(ba.BAError) as e:
            ba.problem_set_tuning(pb, bad)
        assert e.value.status == -1
