"""Parity on a member of the scaling sweep (the city law at 10,000 poses on a
25 km x 5 km loop, ~32M raw-sum clusters), in the launch configuration the
scaling benchmark times: FP64 and precision-form evaluations at the initial
poses against the FP64 oracle over the whole problem."""
import numpy as np
import pytest

import scenes.sums as ss
from helpers import build_gpu_sums, cost_floor, grad_rel_err, oracle_clusters_from_sums, rel

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-12     # FP64 path: rounding-order differences only
TOL32 = 1e-5    # precision form (FP32 storage), as on the other scenes


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sweep(orc):
    import torch
    import paper_2608_14266_amd as ba
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    say("scaling: generating the 10000-pose sweep scene")
    sc = ss.city_sweep_scene(10_000)
    say(f"scaling: {sc.n_clusters} clusters; oracle clusters and evaluation")
    cl = oracle_clusters_from_sums(orc, sc)
    ref = orc.evaluate(orc.MM, cl, sc.poses_init)
    return ba, dev, sc, cl, ref


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sweep_eval_matches_oracle(sweep, orc, prec):
    import torch
    ba, dev, sc, cl, (c_ref, g_ref, H_ref, _) = sweep
    P = torch.as_tensor(sc.poses_init, device=dev)
    kw = {} if prec == "f64" else dict(precision=ba.PREC_F32, ref_poses=P)
    say(f"scaling: {prec} build and eval at the initial poses")
    prob = build_gpu_sums(ba, sc, dev, **kw)
    try:
        ba.tuned(prob, P, cache_path=None, reps=1)
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
        c = float(cost.cpu().numpy()[0])
        g = g.cpu().numpy().ravel()
        H = H.cpu().numpy()
    finally:
        prob.close()
    if prec == "f64":
        assert abs(c - c_ref) <= TOL * c_ref + cost_floor(orc, cl, sc.poses_init)
        assert grad_rel_err(g, g_ref, np.abs(g_ref).sum()) <= TOL
        assert rel(H, H_ref) <= TOL
    else:
        # at the perturbed initial poses the gradient does not cancel, so its
        # error is taken against its own norm
        ec = abs(c - c_ref) / c_ref
        eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
        eH = rel(H, H_ref)
        print(f"  sweep 10000 f32: residual {ec:.2e}  gradient {eg:.2e}  Hessian {eH:.2e}")
        assert ec <= TOL32 and eg <= TOL32 and eH <= TOL32


def test_wide_window_lm_matches_oracle(orc):
    """A single window wider than one solve block's pose rounds (1500 poses)
    runs the increment solve as a statistics launch plus a pose-parallel
    launch; its LM run must follow the oracle's like the narrow windows do."""
    import torch
    import paper_2608_14266_amd as ba
    from helpers import resolved_prefix
    dev = torch.device("cuda:0")
    sc = ss.city_sweep_scene(1500, planes_per_pose=40, seed=5100)
    say(f"scaling: wide window, {sc.n_clusters} clusters; oracle LM")
    cl = oracle_clusters_from_sums(orc, sc)
    P_ref, rep_ref, c_ref = orc.lm(orc.MM, cl, sc.poses_init, 12)
    prob = build_gpu_sums(ba, sc, dev)
    try:
        P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
        reps, tr = ba.iterate(prob, P, ba.MODE_MM, max_iters=12)
    finally:
        prob.close()
    tr = tr[:, 0, :]
    k = resolved_prefix(tr, rep_ref)
    say(f"scaling: wide window, {k} resolved iterations")
    assert k >= 6
    assert np.array_equal(tr[:k, 4], rep_ref[:k, 4])
    assert np.all(np.abs(tr[:k, [0, 1]] - rep_ref[:k, [0, 1]]) <= TOL * np.abs(rep_ref[:k, [0, 1]]))
    # past the resolved prefix rounding decides: 1e-12, or ten times the
    # oracle's own spread under one-ulp perturbations of the start
    from helpers import lm_rounding_spread
    _, dc, dPs = lm_rounding_spread(orc, orc.MM, cl, sc.poses_init, 12)
    print(f"  wide window: final cost error {abs(reps[0]['cost_final'] - c_ref) / c_ref:.2e}, "
          f"oracle spread {dc / c_ref:.2e}, pose spread {dPs.max():.2e}")
    assert abs(reps[0]["cost_final"] - c_ref) <= max(TOL * c_ref, 10 * dc)
    dP = np.abs(P.cpu().numpy() - P_ref)
    assert np.all(dP <= np.maximum(1e-11 * (1.0 + np.abs(P_ref)), 10 * dPs))
