"""The allocation-free increment solve (static device scratch) against the
workspace form of the same solve, through the C-ABI: bitwise equal results on
two calls in a row, the second with a smaller input (the scratch then holds
the first call's data), in the MM and the coupled mode; a size beyond the
static scratch is refused before any device work."""
import ctypes as ct

import numpy as np
import pytest

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


def _mm_system(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, 6, 6))
    H = np.einsum("nij,nkj->nik", A, A) + np.eye(6)[None] * rng.uniform(0.1, 1.0, (n, 1, 1))
    return H, rng.standard_normal(6 * n)


def _dense_system(n_scans, seed):
    rng = np.random.default_rng(seed)
    n = 6 * n_scans
    Q = rng.standard_normal((n, n))
    return Q @ Q.T / n + np.diag(rng.uniform(0.5, 2.0, n)), rng.standard_normal(n)


@pytest.mark.parametrize("mode,sizes", [("mm", (5000, 333)), ("coupled", (500, 137))])
def test_noalloc_solve_equals_workspace_solve(ba, mode, sizes):
    import torch
    dev = torch.device("cuda:0")
    m = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    for k, n in enumerate(sizes):
        say(f"no-alloc solve {mode} n_scans={n} (call {k + 1})")
        H, g = _mm_system(n, 7 + k) if mode == "mm" else _dense_system(n, 7 + k)
        Hd, gd = torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev)
        for mu in (0.0, 0.05):
            dx_ref, info_ref = ba.solve_increment(m, Hd, gd, mu)
            dx, info = ba.solve_increment_noalloc(m, Hd, gd, mu)
            torch.cuda.synchronize()
            assert int(info.cpu().numpy()[0]) == int(info_ref.cpu().numpy()[0]) == 0
            assert np.array_equal(dx.cpu().numpy(), dx_ref.cpu().numpy())


def test_noalloc_reports_a_failing_pivot_like_the_workspace_form(ba):
    import torch
    dev = torch.device("cuda:0")
    H, g = _dense_system(40, 3)
    H[100, :] = 0.0
    H[:, 100] = 0.0
    H[100, 100] = -1.0
    Hd, gd = torch.as_tensor(H, device=dev), torch.as_tensor(g, device=dev)
    dx_ref, info_ref = ba.solve_increment(ba.MODE_COUPLED, Hd, gd, 0.0)
    dx, info = ba.solve_increment_noalloc(ba.MODE_COUPLED, Hd, gd, 0.0)
    assert int(info.cpu().numpy()[0]) == int(info_ref.cpu().numpy()[0]) == 101
    assert np.array_equal(dx.cpu().numpy(), dx_ref.cpu().numpy()) and np.all(dx.cpu().numpy() == 0)


def test_noalloc_refuses_sizes_beyond_the_scratch(ba):
    lib = ba.load()
    ws = lib.ba_solve_increment_workspace(ba.MODE_COUPLED, 1000)
    assert ws > 80 << 20
    one = ct.c_void_p(8)   # never dereferenced: the size check comes first
    st = lib.ba_solve_increment_noalloc(ba.MODE_COUPLED, 1000, one, one, 0.1, one, one, None)
    assert st == -2
    assert b"static scratch" in lib.ba_last_error()
