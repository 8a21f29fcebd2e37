"""Full-size parity on the single-window workload the benchmark times
(500 scans, 200k voxels, ~0.79M clusters from ~117M points), in the same
launch configuration (default build options, MM mode, 20 LM iterations).
The oracle is fast enough here to compare every output, not a sample."""
import numpy as np
import pytest

import scenes
from helpers import block_err_g, block_err_h, cost_floor, grad_rel_err, rel, resolved_prefix, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-12


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def full(orc):
    import torch
    from paper_2608_14266_amd import build as hb
    import os
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2608_14266_amd as ba
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    say("full-size: generating the window scene")
    sc = scenes.window_config(seed=2000)
    say(f"full-size: {sc.n_points} points; oracle clusters")
    cl = orc.scene_clusters(sc)
    say("full-size: GPU build")
    x, y, z, s, v = to_dev(sc, dev)
    prob = ba.build_clusters(x, y, z, s, v, sc.n_scans, sc.n_voxels)
    del x, y, z, s, v
    return ba, dev, sc, cl, prob


def test_fullsize_clusters(full):
    ba, dev, sc, cl, prob = full
    say("full-size clusters")
    vox, scan, cnt, mu, S = [t.cpu().numpy() for t in prob.export_clusters()]
    assert np.array_equal(vox, cl.vox) and np.array_equal(scan, cl.scan)
    assert np.array_equal(cnt, cl.n.astype(np.float64))
    assert np.all(np.abs(mu - cl.mu) <= 4e-16 * np.maximum(np.abs(cl.mu), 1.0))
    assert np.all(np.abs(S - cl.S) <= 1e-13 * np.abs(cl.S).max(axis=1, keepdims=True))


def test_fullsize_eval(full, orc):
    import torch
    ba, dev, sc, cl, prob = full
    say("full-size eval MM at the initial poses")
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sc.poses_init)
    assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref + cost_floor(orc, cl, sc.poses_init)
    assert grad_rel_err(g.cpu().numpy().ravel(), g_ref, np.abs(g_ref).sum()) <= TOL
    assert rel(H.cpu().numpy(), H_ref) <= TOL
    eg, eh = block_err_g(g.cpu().numpy(), g_ref, ga), block_err_h(H.cpu().numpy(), H_ref, Ha)
    print(f"  full size: worst gradient block {eg:.2e}, Hessian block {eh:.2e}")
    assert eg <= TOL and eh <= TOL


def test_fullsize_lm(full, orc):
    import torch
    ba, dev, sc, cl, prob = full
    say("full-size LM, 20 iterations")
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(prob, P, ba.MODE_MM, max_iters=20)
    P_ref, rep_ref, c_ref = orc.lm(orc.MM, cl, sc.poses_init, 20)
    tr = tr[:, 0, :]
    k = resolved_prefix(tr, rep_ref)
    assert k >= 10
    assert np.array_equal(tr[:k, 4], rep_ref[:k, 4])
    assert np.all(np.abs(tr[:k, [0, 1]] - rep_ref[:k, [0, 1]]) <= TOL * np.abs(rep_ref[:k, [0, 1]]))
    assert abs(reps[0]["cost_final"] - c_ref) <= TOL * c_ref
    dP = np.abs(P.cpu().numpy() - P_ref)
    ptol = 1e-11 if k == 20 else 1e-8
    assert np.all(dP <= ptol * (1.0 + np.abs(P_ref)))
