"""ba_iterate runs as one captured HIP graph, replayed while its arguments are
unchanged.  Every replay, with eager work and synchronizations in between,
must reproduce the eager (uncaptured) run bit for bit."""
import os

import numpy as np
import pytest

import scenes
from helpers import build_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode_name", ["MM", "COUPLED"])
def test_graph_replays_match_eager(orc, mode_name):
    import torch
    import paper_2608_14266_amd as ba
    from paper_2608_14266_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mode = getattr(ba, f"MODE_{mode_name}")
    print(f"[gpu-case] graph replay {mode_name}", flush=True)
    sc = scenes.scaled_window(seed=2005, n_scans=30, n_planes=1200)
    prob = build_gpu(ba, sc, dev)
    P0 = torch.as_tensor(sc.poses_init, device=dev)
    os.environ["BA_NO_GRAPH"] = "1"
    try:
        P = P0.clone().contiguous()
        rep_e, tr_e = ba.iterate(prob, P, mode, max_iters=8)
        P_e = P.cpu().numpy().copy()
    finally:
        os.environ.pop("BA_NO_GRAPH", None)
    P = P0.clone().contiguous()
    for replay in range(4):
        P.copy_(P0)
        rep_g, tr_g = ba.iterate(prob, P, mode, max_iters=8)
        assert np.array_equal(P.cpu().numpy(), P_e), replay
        assert np.array_equal(tr_g, tr_e), replay
        assert rep_g == rep_e, replay
        # eager work and a synchronization between replays
        cost, g, H, _ = ba.eval_residual_grad_hessian(prob, P0, ba.MODE_MM)
        torch.cuda.synchronize()
        assert np.isfinite(cost.cpu().numpy()).all()
