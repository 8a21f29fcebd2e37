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
