"""GPU parity of the coupled form: pose-pair Hessian blocks assembled into the
dense per-window matrix, the blocked Cholesky on FP64 matrix cores, and LM
iterations, against the FP64 oracle (and LAPACK for the factorization)."""
import numpy as np
import pytest

import scenes
from helpers import (block_err_g, block_err_h, build_gpu, cost_floor, grad_rel_err, lm_rounding_spread, rel,
                     resolved_prefix)

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


SCENES = {
    "tiny": lambda: scenes.tiny_config(seed=1000, shuffle=True),
    "window-60": lambda: scenes.scaled_window(seed=2001, n_scans=60, n_planes=3000),
    "window-25-ragged": lambda: scenes.scaled_window(seed=2003, n_scans=25, n_planes=900),
}


@pytest.fixture(scope="module", params=list(SCENES))
def case(request, orc):
    sc = SCENES[request.param]()
    return request.param, sc, orc.scene_clusters(sc)


def test_coupled_hessian_matches_oracle(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"coupled eval {name}")
    prob = build_gpu(ba, sc, dev)
    for poses in (sc.poses_init, sc.poses_true):
        P = torch.as_tensor(poses, device=dev)
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P, ba.MODE_COUPLED)
        c_ref, g_ref, H_ref, ga, Ha = orc.evaluate_abs(orc.COUPLED, cl, poses)
        assert abs(cost.cpu().numpy()[0] - c_ref) <= TOL * c_ref + cost_floor(orc, cl, poses)
        Hg = H.cpu().numpy()
        assert rel(Hg, H_ref) <= TOL
        # every pose-pair block against its own rounding scale
        assert block_err_h(Hg, H_ref, Ha) <= TOL
        assert block_err_g(g.cpu().numpy(), g_ref, ga) <= TOL
        assert np.array_equal(Hg, Hg.T)            # both triangles written from one sum


@pytest.mark.parametrize("n", [6, 60, 66, 126, 150, 198, 300, 330, 384])
def test_dense_cholesky_solve_against_lapack(ba, dev, orc, n):
    import torch
    say(f"dense solve random SPD n={n}")
    rng = np.random.default_rng(n)
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T / n + np.diag(rng.uniform(0.5, 2.0, n))
    g = rng.standard_normal(n)
    for mu in (0.0, 0.1):
        dx, info = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev),
                                      torch.as_tensor(g, device=dev), mu)
        assert int(info.cpu().numpy()[0]) == 0
        D = np.maximum(np.diag(H), 1e-12 * np.diag(H).max())
        ref = np.linalg.solve(H + mu * np.diag(D), -g)
        cond = np.linalg.cond(H + mu * np.diag(D))
        assert rel(dx.cpu().numpy().ravel(), ref) <= 1e-15 * cond * 10
        ref_o, info_o = orc.solve(orc.COUPLED, n // 6, H, g, mu) if n % 6 == 0 else (None, 0)
        if ref_o is not None:
            assert info_o == 0 and rel(dx.cpu().numpy().ravel(), ref_o) <= 1e-15 * cond * 10


@pytest.mark.parametrize("n", [1026, 4098, 6000, 6144])
def test_dense_solve_large_against_lapack(ba, dev, n):
    """Sizes where the dataflow factorization has many tile rows, with ragged
    last tiles (1026, 4098, 6000) and at its size limit (6144)."""
    import torch
    say(f"dense solve random SPD n={n}")
    rng = np.random.default_rng(n)
    Q = rng.standard_normal((n, 256))
    H = Q @ Q.T / 256 + np.diag(rng.uniform(0.5, 2.0, n))
    g = rng.standard_normal(n)
    dx, info = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), 0.1)
    assert int(info.cpu().numpy()[0]) == 0
    D = np.diag(H)
    A = H + 0.1 * np.diag(D)
    ref = np.linalg.solve(A, -g)
    x = dx.cpu().numpy().ravel()
    # normwise backward error against LAPACK's own on the same system
    be = np.linalg.norm(A @ x + g) / (np.linalg.norm(A, 1) * np.linalg.norm(x) + np.linalg.norm(g))
    be_ref = np.linalg.norm(A @ ref + g) / (np.linalg.norm(A, 1) * np.linalg.norm(ref) + np.linalg.norm(g))
    assert be <= 16 * max(be_ref, np.finfo(float).eps)
    assert rel(x, ref) <= 10 * np.finfo(float).eps * np.linalg.cond(A)


def test_dense_flow_gives_up_when_told(ba, dev, monkeypatch):
    """A wait of the dataflow factorization that gives up (forced from the
    host with a negative poll limit) aborts the launch: the solve reports
    info = -1 with dx = 0, every kernel ends, and the next solve is exact."""
    import torch
    n = 384
    say(f"dense solve abort path n={n}")
    rng = np.random.default_rng(11)
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T / n + np.eye(n)
    g = rng.standard_normal(n)
    Ht, gt = torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev)
    monkeypatch.setenv("BA_FLOW_SPIN", "-1")
    dx, info = ba.solve_increment(ba.MODE_COUPLED, Ht, gt, 0.0)
    assert int(info.cpu().numpy()[0]) == -1
    assert np.all(dx.cpu().numpy() == 0)
    monkeypatch.delenv("BA_FLOW_SPIN")
    dx, info = ba.solve_increment(ba.MODE_COUPLED, Ht, gt, 0.0)
    assert int(info.cpu().numpy()[0]) == 0
    ref = np.linalg.solve(H, -g)
    assert rel(dx.cpu().numpy().ravel(), ref) <= 1e-15 * np.linalg.cond(H) * 10


@pytest.mark.parametrize("n", [90, 198, 384])
def test_dense_solve_reads_lower_triangle_only(ba, dev, n):
    """The coupled solve uses the lower triangle of hess: noise in the strict
    upper triangle (inside and outside the diagonal tiles) leaves dx bitwise
    unchanged."""
    import torch
    say(f"dense solve lower triangle only n={n}")
    rng = np.random.default_rng(7 * n)
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T / n + np.diag(rng.uniform(0.5, 2.0, n))
    g = rng.standard_normal(n)
    Hn = H.copy()
    iu = np.triu_indices(n, 1)
    Hn[iu] = rng.standard_normal(len(iu[0])) * 1e3
    dx1, i1 = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), 0.1)
    dx2, i2 = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(Hn, device=dev), torch.as_tensor(g, device=dev), 0.1)
    assert int(i1.cpu().numpy()[0]) == int(i2.cpu().numpy()[0]) == 0
    assert np.array_equal(dx1.cpu().numpy(), dx2.cpu().numpy())


@pytest.mark.parametrize("bad", [3, 64, 65, 150])
def test_dense_cholesky_reports_pivot(ba, dev, orc, bad):
    import torch
    say(f"dense solve failing pivot at {bad}")
    n = 192
    rng = np.random.default_rng(bad)
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T / n + np.eye(n)
    # make the leading (bad+1) x (bad+1) block indefinite at exactly pivot `bad`
    H[bad, :] = 0.0
    H[:, bad] = 0.0
    H[bad, bad] = -1.0
    g = np.ones(n)
    dx, info = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev), 0.0)
    _, info_o = orc.solve(orc.COUPLED, n // 6, H, g, 0.0)
    assert int(info.cpu().numpy()[0]) == info_o == bad + 1
    assert np.all(dx.cpu().numpy() == 0)


def test_coupled_solve_matches_oracle(ba, dev, orc, case):
    import torch
    name, sc, cl = case
    say(f"coupled solve {name}")
    _, g, H, _ = orc.evaluate(orc.COUPLED, cl, sc.poses_init)
    for mu in (1e-2, 1.0):
        dx, info = ba.solve_increment(ba.MODE_COUPLED, torch.as_tensor(H, device=dev),
                                      torch.as_tensor(g, device=dev), mu)
        ref, info_ref = orc.solve(orc.COUPLED, sc.n_scans, H, g, mu)
        assert int(info.cpu().numpy()[0]) == info_ref == 0
        fl = 1e-12 * np.diag(H).max()
        A = H + mu * np.diag(np.maximum(np.diag(H), fl))
        cond = np.linalg.cond(A)
        assert rel(dx.cpu().numpy().ravel(), ref) <= max(TOL, 1e-15 * cond * 10)


@pytest.mark.parametrize("iters", [10])
def test_iterate_coupled_matches_oracle(ba, dev, orc, case, iters):
    import torch
    name, sc, cl = case
    say(f"iterate coupled {name}")
    prob = build_gpu(ba, sc, dev)
    P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
    reps, tr = ba.iterate(prob, P, ba.MODE_COUPLED, max_iters=iters)
    P_ref, rep_ref, c_ref = orc.lm(orc.COUPLED, cl, sc.poses_init, iters)
    tr = tr[:, 0, :]
    k = resolved_prefix(tr, rep_ref)
    assert k >= 3          # the coupled step is Newton-like: a few resolved iterations
    assert np.array_equal(tr[:k, 4], rep_ref[:k, 4])
    # 1e-12, or ten times the oracle's own spread under one-ulp perturbations
    # of the start where the dense damped solve amplifies rounding beyond it
    dtr, dc, _ = lm_rounding_spread(orc, orc.COUPLED, cl, sc.poses_init, iters)
    scale = np.maximum(np.abs(rep_ref[:k, [0, 1]]), 1e-3 * rep_ref[0, 0])
    tol = np.maximum(TOL * scale, 10 * dtr[:k, 0:2])
    err = np.abs(tr[:k, [0, 1]] - rep_ref[:k, [0, 1]])
    print(f"  {name}: worst trace error / (TOL scale) {np.max(err / (TOL * scale)):.2e}, "
          f"oracle spread / (TOL scale) {np.max(dtr[:k, 0:2] / (TOL * scale)):.2e}")
    assert np.all(err <= tol)
    assert abs(reps[0]["cost_final"] - c_ref) <= max(TOL * max(c_ref, 1e-3 * rep_ref[0, 0]), 10 * dc)


def test_mm_and_coupled_reach_same_minimum(ba, dev, orc):
    import torch
    say("MM vs coupled minimum")
    sc = scenes.tiny_config(seed=1004)
    prob = build_gpu(ba, sc, dev)
    costs = []
    for mode in (ba.MODE_MM, ba.MODE_COUPLED):
        P = torch.as_tensor(sc.poses_init, device=dev).contiguous()
        reps, _ = ba.iterate(prob, P, mode, max_iters=40)
        costs.append(reps[0]["cost_final"])
    assert abs(costs[0] - costs[1]) <= 1e-9 * costs[0]
