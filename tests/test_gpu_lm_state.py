"""GPU tests of the LM state a run reports: the final gradient norm is formed
in the order of the in-loop convergence test (bitwise), and a run resumed
with the reported damping (mu_final, nu_final) continues exactly where it
stopped, for windows wider than one statistics pass (> 512 poses) in both
modes."""
import numpy as np
import pytest

import scenes.sums as ss
from helpers import build_gpu_sums

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ba():
    import os
    import torch
    from paper_2608_14266_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2608_14266_amd as m
    m.load()
    torch.cuda.set_device(torch.device("cuda:0"))
    return m


@pytest.fixture(scope="module")
def wide():
    # one window of 700 poses (wider than the 512-thread statistics order)
    return ss.request_scene(seed=5200, n_poses=700, vox_per_pose=20)


@pytest.mark.parametrize("mode", ["mm", "coupled"])
def test_final_gradient_norm_is_the_in_loop_one(ba, wide, mode):
    """gnorm_final after k iterations equals, bitwise, the gradient norm the
    (k+1)-th iteration's decision records at the same poses."""
    import torch
    dev = torch.device("cuda:0")
    m = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    k = 4 if mode == "mm" else 2
    say(f"final gnorm order {mode}")
    prob = build_gpu_sums(ba, wide, dev)
    try:
        P = torch.as_tensor(wide.poses_init, device=dev).contiguous()
        reps, _ = ba.iterate(prob, P, m, max_iters=k)
        P2 = torch.as_tensor(wide.poses_init, device=dev).contiguous()
        _, tr = ba.iterate(prob, P2, m, max_iters=k + 1)
    finally:
        prob.close()
    assert reps[0]["gnorm_final"] == tr[k, 0, 5]
    assert reps[0]["gnorm_final"] > 0


@pytest.mark.parametrize("mode", ["mm", "coupled"])
def test_resume_with_reported_damping_is_exact(ba, wide, mode):
    import torch
    dev = torch.device("cuda:0")
    m = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    k1, k2 = (5, 4) if mode == "mm" else (2, 2)
    say(f"resume {mode}")
    prob = build_gpu_sums(ba, wide, dev)
    try:
        P = torch.as_tensor(wide.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(prob, P, m, max_iters=k1)
        r2, t2 = ba.iterate(prob, P, m, max_iters=k2, mu0=r1[0]["mu_final"], nu0=r1[0]["nu_final"])
        Q = torch.as_tensor(wide.poses_init, device=dev).contiguous()
        r3, t3 = ba.iterate(prob, Q, m, max_iters=k1 + k2)
    finally:
        prob.close()
    assert r1[0]["nu_final"] >= 2.0
    assert np.array_equal(P.cpu().numpy(), Q.cpu().numpy())
    assert np.array_equal(np.concatenate([t1, t2]), t3)
    assert r2[0]["cost_final"] == r3[0]["cost_final"] and r2[0]["mu_final"] == r3[0]["mu_final"]
    assert r2[0]["nu_final"] == r3[0]["nu_final"] and r2[0]["gnorm_final"] == r3[0]["gnorm_final"]


@pytest.fixture(scope="module")
def three():
    # three windows of 12, 30 and 20 poses in one problem
    return ss.batch_windows(seed=5300, n_windows=3, poses=[12, 30, 20], vox_range=(400, 2000), workers=1)


@pytest.mark.parametrize("mode", ["mm", "coupled"])
def test_per_window_resume_is_exact(ba, three, mode):
    """Chunks resumed per window (each window's own mu, nu and rejection
    count from the previous chunk's report) give the bits of one uninterrupted
    run, for every window of a batched problem."""
    import torch
    dev = torch.device("cuda:0")
    m = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    k1, k2 = (4, 5) if mode == "mm" else (2, 3)
    say(f"per-window resume {mode}")
    prob = build_gpu_sums(ba, three, dev)
    try:
        P = torch.as_tensor(three.poses_init, device=dev).contiguous()
        r1, t1 = ba.iterate(prob, P, m, max_iters=k1, max_rejects=3)
        res = np.array([[r["mu_final"], r["nu_final"], r["rejects_final"], 0.0] for r in r1])
        r2, t2 = ba.iterate(prob, P, m, max_iters=k2, max_rejects=3, resume=res)
        Q = torch.as_tensor(three.poses_init, device=dev).contiguous()
        r3, t3 = ba.iterate(prob, Q, m, max_iters=k1 + k2, max_rejects=3)
    finally:
        prob.close()
    assert np.array_equal(P.cpu().numpy(), Q.cpu().numpy())
    assert np.array_equal(np.concatenate([t1, t2]), t3)
    for a, b in zip(r2, r3):
        for k in ("cost_final", "gnorm_final", "mu_final", "nu_final", "rejects_final", "converged", "stalled"):
            assert a[k] == b[k], k


def test_skipped_window_is_left_alone(ba, three):
    """A window skipped through the per-window start keeps its poses and runs
    no iteration; the other windows are bitwise what they are without the skip."""
    import torch
    dev = torch.device("cuda:0")
    say("skipped window")
    prob = build_gpu_sums(ba, three, dev)
    try:
        base = np.array([[1e-2, 2.0, 0.0, 0.0]] * 3)
        P = torch.as_tensor(three.poses_init, device=dev).contiguous()
        ra, _ = ba.iterate(prob, P, ba.MODE_MM, max_iters=6, resume=base)
        skip = base.copy()
        skip[1, 3] = 1.0
        Q = torch.as_tensor(three.poses_init, device=dev).contiguous()
        rb, _ = ba.iterate(prob, Q, ba.MODE_MM, max_iters=6, resume=skip)
        # per-window start equal to the scalar defaults gives the default run
        R = torch.as_tensor(three.poses_init, device=dev).contiguous()
        rc, _ = ba.iterate(prob, R, ba.MODE_MM, max_iters=6)
        with pytest.raises(ba.BAError):
            bad = base.copy()
            bad[2, 0] = 0.0
            ba.iterate(prob, R, ba.MODE_MM, max_iters=1, resume=bad)
    finally:
        prob.close()
    sw = three.scan_window
    P, Q, R = P.cpu().numpy(), Q.cpu().numpy(), R.cpu().numpy()
    w1 = sw == 1
    assert np.array_equal(Q[w1], three.poses_init[w1])
    assert rb[1]["iters"] == 0
    assert np.array_equal(Q[~w1], P[~w1])
    for w in (0, 2):
        assert rb[w] == ra[w]
    assert np.array_equal(P, R) and ra == rc
