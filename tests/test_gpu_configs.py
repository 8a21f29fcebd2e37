"""Oracle parity on the paths the benchmark workloads actually take, at their
real shapes:

  * the dense Cholesky solve at the single-window size (n = 6 x 500 = 3000,
    47 diagonal blocks: an odd block count) and the city size
    (n = 6 x 2000 = 12000), against LAPACK;
  * the coupled evaluation and one damped coupled solve on the full
    500-pose window against the oracle;
  * the single-window evaluation in the launch configuration the benchmark
    times (the autotuner's choices), against the oracle;
  * a batch shaped like the 256-window workload (16 windows, poses per window
    log-uniform in [20, 400], 200 voxels per pose clipped to [5k, 80k]), per
    window, in FP64 and in the precision form.

Gradients and Hessians are compared per pose block, each block against its
own rounding scale (oracle.evaluate_abs), at 1e-12 (FP64) and 1e-5 (FP32)."""
import numpy as np
import pytest

import scenes
import scenes.sums as ss
from helpers import (block_err_g, block_err_h, build_gpu_sums, cost_floor, dense_backward_error,
                     oracle_clusters_from_sums, rel, to_dev)

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-12
TOL32 = 1e-5
EPS = np.finfo(np.float64).eps


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
def window(ba, orc):
    import torch
    dev = torch.device("cuda:0")
    say("configs: generating the 500-pose window scene")
    sc = scenes.window_config(seed=2000)
    cl = orc.scene_clusters(sc)
    x, y, z, s, v = to_dev(sc, dev)
    prob = ba.build_clusters(x, y, z, s, v, sc.n_scans, sc.n_voxels)
    del x, y, z, s, v
    yield dev, sc, cl, prob
    prob.close()


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    return Q @ Q.T / n + np.diag(rng.uniform(0.5, 2.0, n)), rng.standard_normal(n)


@pytest.mark.parametrize("n", [3000, 12000])
def test_dense_solve_at_workload_sizes_against_lapack(ba, n):
    """Block counts 47 (odd: the two-row back-substitution ends with a single
    row) and 188.  The backward error of the GPU solution must be within 16x
    LAPACK's own on the same system; where LAPACK's condition estimate is
    affordable (n = 3000) the solution also agrees to 10 eps kappa."""
    import torch
    dev = torch.device("cuda:0")
    say(f"dense solve n={n}")
    H, g = _spd(n, n)
    for mu in (0.0, 0.1):
        dx, info = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev),
                                      torch.as_tensor(g, device=dev), mu)
        assert int(info.cpu().numpy()[0]) == 0
        D = np.maximum(np.diag(H), 1e-12 * np.diag(H).max())
        A = H + mu * np.diag(D)
        ref = np.linalg.solve(A, -g)
        x = dx.cpu().numpy().ravel()
        be, be_ref = dense_backward_error(A, x, -g), dense_backward_error(A, ref, -g)
        print(f"  n={n} mu={mu}: backward error gpu {be:.2e} lapack {be_ref:.2e}")
        assert be <= 16 * max(be_ref, EPS)
        if n <= 3000:
            cond = np.linalg.cond(A)
            assert rel(x, ref) <= 10 * EPS * cond
        del A
    # deterministic
    dx2, _ = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), 0.1)
    assert np.array_equal(dx2.cpu().numpy(), dx.cpu().numpy())


def test_window_coupled_eval_and_solve_match_oracle(ba, orc, window):
    import torch
    dev, sc, cl, prob = window
    say("configs: coupled eval on the 500-pose window")
    P = torch.as_tensor(sc.poses_init, device=dev)
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_COUPLED)
    c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.COUPLED, cl, sc.poses_init)
    c = float(cost.cpu().numpy()[0])
    g = g.cpu().numpy().ravel()
    Hg = H.cpu().numpy()
    eg, eh = block_err_g(g, g_ref, ga), block_err_h(Hg, H_ref, Ha)
    print(f"  coupled window: cost {abs(c - c_ref) / c_ref:.2e}  grad block {eg:.2e}  hess block {eh:.2e}")
    assert abs(c - c_ref) <= TOL * c_ref
    assert eg <= TOL and eh <= TOL
    assert np.array_equal(Hg, Hg.T)
    # one damped coupled solve (the step of the first LM iteration).  The GPU
    # factorization on the oracle's matrix isolates the solve: 10 eps kappa;
    # the GPU chain (its own H and g) adds their 1e-12 block errors, amplified
    # by kappa.
    mu = 1e-2
    fl = 1e-12 * np.diag(H_ref).max()
    A = H_ref + mu * np.diag(np.maximum(np.diag(H_ref), fl))
    cond = np.linalg.cond(A)
    ref, info_ref = orc.solve(orc.COUPLED, sc.n_scans, H_ref, g_ref, mu)
    assert info_ref == 0
    dx_o, info_o = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H_ref, device=dev),
                                      torch.as_tensor(g_ref, device=dev), mu)
    dx_g, info_g = ba.solve_increment(ba.MODE_COUPLED, H, torch.as_tensor(g, device=dev), mu)
    assert int(info_o.cpu().numpy()[0]) == 0 and int(info_g.cpu().numpy()[0]) == 0
    e_solve = rel(dx_o.cpu().numpy().ravel(), ref)
    e_chain = rel(dx_g.cpu().numpy().ravel(), ref)
    print(f"  coupled window solve: kappa {cond:.2e}, solve {e_solve:.2e}, chain {e_chain:.2e}")
    assert e_solve <= 10 * EPS * cond
    assert e_chain <= (TOL + 10 * EPS) * cond


def test_window_eval_autotuned_matches_oracle(ba, orc, window):
    """The launch choices the benchmark applies (autotuned) against the oracle."""
    import torch
    dev, sc, cl, prob = window
    P = torch.as_tensor(sc.poses_init, device=dev)
    t = ba.tuned(prob, P, cache_path=None, reps=3)
    say(f"configs: autotuned window eval {t}")
    cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_MM)
    c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sc.poses_init)
    c = float(cost.cpu().numpy()[0])
    eg = block_err_g(g.cpu().numpy(), g_ref, ga)
    eh = block_err_h(H.cpu().numpy(), H_ref, Ha)
    print(f"  autotuned window: cost {abs(c - c_ref) / c_ref:.2e}  grad block {eg:.2e}  hess block {eh:.2e}")
    assert abs(c - c_ref) <= TOL * c_ref + cost_floor(orc, cl, sc.poses_init)
    assert eg <= TOL and eh <= TOL


@pytest.fixture(scope="module")
def batch16():
    # the 256-window law (poses log-uniform [20, 400], clip(200 N_w, 5k, 80k)
    # voxels), 16 windows of it
    return ss.batch_windows(seed=4300, n_windows=16)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_shaped_windows_match_oracle(ba, orc, batch16, prec):
    import torch
    dev = torch.device("cuda:0")
    sc = batch16
    say(f"configs: 16-window batch {prec}, {sc.n_clusters} clusters, poses {sc.meta['poses']}")
    P = torch.as_tensor(sc.poses_init, device=dev)
    kw = {} if prec == "f64" else dict(precision=ba.PREC_F32, ref_poses=P)
    pb = build_gpu_sums(ba, sc, dev, **kw)
    try:
        ba.tuned(pb, P, cache_path=None, reps=2)
        cost, g, H, _ = ba.eval_residual_grad_hessian(pb, P, ba.MODE_MM)
        cost = cost.cpu().numpy()
        g = g.cpu().numpy().reshape(-1, 6)
        H = H.cpu().numpy()
    finally:
        pb.close()
    tol = TOL if prec == "f64" else TOL32
    worst = [0.0, 0.0, 0.0]
    s0 = 0
    for w in range(sc.n_windows):
        sw = ss.window_of(sc, w)
        cl = oracle_clusters_from_sums(orc, sw)
        c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.MM, cl, sw.poses_init)
        n = sw.n_scans
        e = (abs(cost[w] - c_ref) / c_ref, block_err_g(g[s0:s0 + n], g_ref, ga),
             block_err_h(H[s0:s0 + n], H_ref, Ha))
        worst = [max(a, b) for a, b in zip(worst, e)]
        assert e[0] <= tol and e[1] <= tol and e[2] <= tol, (w, e)
        s0 += n
    print(f"  batch {prec}: worst residual {worst[0]:.2e}  grad block {worst[1]:.2e}  hess block {worst[2]:.2e}")
