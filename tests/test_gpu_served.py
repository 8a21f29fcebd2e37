"""GPU tests of the served form: the request server admits window problems
by device-memory budget into concurrent slots and solves each to the
gradient tolerance.

Bar: every request's result (poses and LM report) is bitwise identical
whether it is served alone or in a mix of concurrent requests; served
results agree with the oracle's own LM run with the same options (cost and
poses at 1e-12, or at ten times the oracle's rounding spread where rounding
decides the late steps);
the footprint used for admission bounds the real device memory; a budget
that fits one request at a time serialises the requests."""
import numpy as np
import pytest

import scenes.sums as ss
from helpers import build_gpu_sums, oracle_clusters_from_sums

pytestmark = pytest.mark.gpu


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
def requests():
    sizes = [12, 30, 8, 45, 20, 16, 60, 10]
    return [ss.request_scene(seed=5000 + i, n_poses=n, vox_per_pose=40) for i, n in enumerate(sizes)]


GB = 1 << 30


def _serve(ba, reqs, slots, budget, **kw):
    with ba.Server(budget, slots=slots, **kw) as srv:
        ids = [srv.submit_scene(r) for r in reqs]
        return [srv.wait(i) for i in ids]


@pytest.mark.parametrize("prec,mode", [("f64", "mm"), ("f32", "mm"), ("f64", "coupled")])
def test_each_result_is_the_same_alone_and_in_the_mix(ba, dev, requests, prec, mode):
    say(f"served alone vs mix {prec} {mode}")
    kw = dict(precision=ba.PREC_F64 if prec == "f64" else ba.PREC_F32,
              mode=ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED,
              max_iters=30 if mode == "mm" else 12, tol_g=1e-6)
    alone = [_serve(ba, [r], 1, 8 * GB, **kw)[0] for r in requests]
    mix = _serve(ba, requests, 4, 8 * GB, **kw)
    overlap = 0
    for (pa, sa), (pm, sm) in zip(alone, mix):
        assert sa["state"] == sm["state"] == ba._lib.REQ_DONE
        assert np.array_equal(pa, pm)
        assert sa["report"] == sm["report"]
    # the mix really ran requests side by side
    iv = sorted((s["t_admit"], s["t_done"]) for _, s in mix)
    overlap = sum(1 for a, b in zip(iv, iv[1:]) if b[0] < a[1])
    print(f"  {prec}/{mode}: {overlap} overlapping admissions")
    assert overlap >= 1


@pytest.mark.parametrize("mode", ["mm", "coupled"])
def test_served_results_match_oracle_lm(ba, dev, orc, requests, mode):
    """Each served request against the oracle's own LM run with the same
    options (gradient tolerance 1e-6, 10 rejections in a row stop a request):
    final cost and poses to 1e-12, or ten times the oracle's own spread under
    one-ulp perturbations of the start once rounding decides the late steps;
    the iteration and acceptance counts where the oracle's perturbed runs agree
    on them.  The coupled form reaches the gradient tolerance; the MM form on
    these chain-like windows does not within the cap (its block-diagonal step
    leaves the slow along-chain modes: see the design notes)."""
    from helpers import lm_rounding_spread
    say(f"served vs oracle LM ({mode})")
    m_ba = ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED
    m_orc = orc.MM if mode == "mm" else orc.COUPLED
    iters = 40 if mode == "mm" else 25
    res = _serve(ba, requests[:4], 4, 8 * GB, mode=m_ba, max_iters=iters, tol_g=1e-6, max_rejects=10)
    for i, (r, (P, st)) in enumerate(zip(requests[:4], res)):
        cl = oracle_clusters_from_sums(orc, r)
        P_ref, rep_ref, c_ref = orc.lm(m_orc, cl, r.poses_init, iters, tol_g=1e-6, max_rejects=10)
        dtr, dc, dP = lm_rounding_spread(orc, m_orc, cl, r.poses_init, iters, tol_g=1e-6, max_rejects=10)
        rep = st["report"]
        ec = abs(rep["cost_final"] - c_ref)
        ep = np.abs(P - P_ref)
        print(f"  request {i} ({r.n_scans} poses): cost err {ec / c_ref:.2e} (spread {dc / c_ref:.2e}), "
              f"pose err {ep.max():.2e} (spread {dP.max():.2e}), iters {rep['iters']} / {len(rep_ref)}, "
              f"gnorm {rep['gnorm_final']:.2e}")
        assert ec <= max(1e-12 * c_ref, 10 * dc)
        assert np.all(ep <= np.maximum(1e-11 * (1.0 + np.abs(P_ref)), 10 * dP))
        if dc == 0.0 and not np.any(dP):
            # the oracle's iteration does not depend on rounding here
            assert rep["iters"] == len(rep_ref)
            assert rep["n_accepted"] == int(rep_ref[:, 4].sum())
        assert rep["cost_final"] < rep["cost_initial"]
        if mode == "coupled":
            assert rep["converged"] == 1 and rep["gnorm_final"] < 1e-6


def test_budget_of_one_request_serialises(ba, dev, requests):
    say("tiny budget")
    fp = [ba.request_footprint(r.voxel, r.scan, r.count, r.sum, r.sumsq, r.n_scans, r.n_voxels, r.poses_init)
          for r in requests]
    budget = max(fp)            # fits any single request, never two of the largest
    res = _serve(ba, requests, 4, budget, max_iters=10, tol_g=0.0)
    iv = sorted((s["t_admit"], s["t_done"], s["footprint"]) for _, s in res)
    # at every admission the reserved bytes stay within the budget
    for a in iv:
        live = sum(f for (s0, s1, f) in iv if s0 <= a[0] < s1)
        assert live <= budget
    alone = [_serve(ba, [r], 1, 8 * GB, max_iters=10, tol_g=0.0)[0] for r in requests]
    for (pa, _), (pm, _) in zip(alone, res):
        assert np.array_equal(pa, pm)


def test_footprint_bounds_device_memory(ba, dev, requests):
    import torch
    say("footprint bound")
    for r in requests[:3]:
        for mode in (ba.MODE_MM, ba.MODE_COUPLED):
            for prec in (ba.PREC_F64, ba.PREC_F32):
                fp = ba.request_footprint(r.voxel, r.scan, r.count, r.sum, r.sumsq, r.n_scans, r.n_voxels,
                                          r.poses_init, mode=mode, precision=prec)
                kw = {} if prec == ba.PREC_F64 else dict(precision=prec,
                                                          ref_poses=torch.as_tensor(r.poses_init, device=dev))
                p = build_gpu_sums(ba, r, dev, **kw)
                P = torch.as_tensor(r.poses_init, device=dev).contiguous()
                ba.iterate(p, P, mode, max_iters=2)
                used = p.info()["device_bytes"]
                assert used <= fp, (mode, prec, used, fp)


def test_over_budget_request_is_refused(ba, dev, requests):
    with ba.Server(1 << 20, slots=2) as srv:
        with pytest.raises(ba.BAError) as e:
            srv.submit_scene(requests[0])
        assert e.value.status == -7


def test_unknown_request_id(ba, dev):
    with ba.Server(GB, slots=1) as srv:
        with pytest.raises(ba.BAError) as e:
            srv.query(12345)
        assert e.value.status == -8


def test_chunked_lm_does_not_change_results(ba, dev, requests):
    """The served LM runs in chunks of iters_per_check iterations that resume
    each other exactly: every chunk length gives the same bits."""
    say("served chunk lengths")
    outs = []
    for k in (1, 3, 0):
        res = _serve(ba, requests[:3], 2, 8 * GB, max_iters=12, tol_g=1e-6, max_rejects=3, iters_per_check=k)
        outs.append(res)
    for res in outs[1:]:
        for (pa, sa), (pb, sb) in zip(outs[0], res):
            assert np.array_equal(pa, pb)
            assert sa["report"] == sb["report"]


def test_cancel_leaves_the_other_requests_unchanged(ba, dev, requests):
    """Cancelling a running request (mid-run) and a queued one: both end
    cancelled; every other request's poses and report are bitwise those it
    gets served alone."""
    import time
    say("served cancel")
    kw = dict(max_iters=400, tol_g=0.0, max_rejects=0, iters_per_check=1)
    long_kw = dict(kw, max_iters=4000)
    long_req = ss.request_scene(seed=5100, n_poses=300, vox_per_pose=60)
    others = requests[:4]
    # the long request's server runs 4000 iterations per request; the others
    # are compared with their own 400-iteration runs alone, so they are served
    # by a second server at the same time (both share the GPU)
    with ba.Server(8 * GB, slots=1, **long_kw) as srv_long, ba.Server(8 * GB, slots=2, **kw) as srv:
        rid_long = srv_long.submit_scene(long_req)
        ids = [srv.submit_scene(r) for r in others]
        rid_queued = srv.submit_scene(requests[4])
        # the queued one: cancelled before any slot takes it
        srv.cancel(rid_queued)
        t0 = time.time()
        while srv_long.query(rid_long)["state"] != ba._lib.REQ_RUNNING and time.time() - t0 < 60:
            time.sleep(0.001)
        time.sleep(0.2)   # let it run a number of iterations first
        srv_long.cancel(rid_long)
        P_long, st_long = srv_long.wait_any(rid_long)
        P_q, st_q = srv.wait_any(rid_queued)
        res = [srv.wait(i) for i in ids]
    assert st_q["state"] == ba._lib.REQ_CANCELLED and st_q["report"]["iters"] == 0
    assert np.array_equal(P_q, requests[4].poses_init)
    assert st_long["state"] == ba._lib.REQ_CANCELLED
    assert 0 < st_long["report"]["iters"] < long_kw["max_iters"]
    assert st_long["report"]["cost_final"] < st_long["report"]["cost_initial"]
    print(f"  cancelled the long request after {st_long['report']['iters']} iterations")
    alone = [_serve(ba, [r], 1, 8 * GB, **kw)[0] for r in others]
    for (pa, sa), (pm, sm) in zip(alone, res):
        assert sm["state"] == ba._lib.REQ_DONE
        assert np.array_equal(pa, pm)
        assert sa["report"] == sm["report"]
    with ba.Server(GB, slots=1) as srv:
        with pytest.raises(ba.BAError) as e:
            srv.cancel(777)
        assert e.value.status == -8


def _blocked_serve(ba, reqs, budget, **kw):
    """Serve `reqs` on one slot behind a long blocker request, so that they
    are all queued when the slot takes them (batches form deterministically)."""
    import time
    blocker = ss.request_scene(seed=5102, n_poses=1000, vox_per_pose=100)
    with ba.Server(budget, slots=1, **kw) as srv:
        rb = srv.submit_scene(blocker)
        t0 = time.time()
        while srv.query(rb)["state"] == ba._lib.REQ_QUEUED and time.time() - t0 < 60:
            time.sleep(0.001)
        ids = [srv.submit_scene(r) for r in reqs]
        assert srv.query(rb)["state"] == ba._lib.REQ_RUNNING, "the blocker ended before the requests were queued"
        out = [srv.wait_any(i) for i in ids]
        srv.wait(rb)
    return out


@pytest.mark.parametrize("prec,mode", [("f32", "mm"), ("f64", "coupled")])
def test_batched_admission_equals_alone(ba, dev, requests, prec, mode):
    """A slot that fuses up to four queued requests into one problem of
    windows gives every request the poses and report it gets served alone
    (each window resumes its own run at every chunk and stops on its own)."""
    say(f"served batched admission {prec} {mode}")
    kw = dict(precision=ba.PREC_F64 if prec == "f64" else ba.PREC_F32,
              mode=ba.MODE_MM if mode == "mm" else ba.MODE_COUPLED,
              max_iters=30 if mode == "mm" else 12, tol_g=1e-6, max_rejects=10, iters_per_check=3)
    alone = [_serve(ba, [r], 1, 8 * GB, **kw)[0] for r in requests]
    fused = _blocked_serve(ba, requests, 8 * GB, batch=4, **kw)
    for (pa, sa), (pb, sb) in zip(alone, fused):
        assert sa["state"] == sb["state"] == ba._lib.REQ_DONE
        assert np.array_equal(pa, pb)
        assert sa["report"] == sb["report"]
    # the eight queued requests went in two batches of four
    admits = [s["t_admit"] for _, s in fused]
    assert len(set(admits)) == 2 and admits.count(admits[0]) == 4
    # each request finished when its own window stopped, not with its batch
    done = [s["t_done"] for _, s in fused]
    print(f"  {prec}/{mode}: distinct completion times {len(set(done))} of {len(done)}")


def test_cancel_inside_a_batch(ba, dev, requests):
    """Cancelling one request of a running batch: it ends cancelled with the
    poses it reached; the other requests of the batch are bitwise those they
    get served alone."""
    import time
    say("served cancel inside a batch")
    kw = dict(max_iters=400, tol_g=0.0, max_rejects=0, iters_per_check=1)
    reqs = requests[:4]
    alone = [_serve(ba, [r], 1, 8 * GB, **kw)[0] for r in reqs]
    blocker = ss.request_scene(seed=5103, n_poses=600, vox_per_pose=60)
    with ba.Server(8 * GB, slots=1, batch=4, **kw) as srv:
        rb = srv.submit_scene(blocker)
        t0 = time.time()
        while srv.query(rb)["state"] == ba._lib.REQ_QUEUED and time.time() - t0 < 60:
            time.sleep(0.001)
        ids = [srv.submit_scene(r) for r in reqs]
        while srv.query(ids[2])["state"] != ba._lib.REQ_RUNNING and time.time() - t0 < 60:
            time.sleep(0.001)
        time.sleep(0.02)
        srv.cancel(ids[2])
        res = [srv.wait_any(i) for i in ids]
        srv.wait(rb)
    Pc, sc_ = res[2]
    assert sc_["state"] == ba._lib.REQ_CANCELLED
    assert 0 < sc_["report"]["iters"] < 400
    assert not np.array_equal(Pc, reqs[2].poses_init)
    for k in (0, 1, 3):
        assert res[k][1]["state"] == ba._lib.REQ_DONE
        assert np.array_equal(res[k][0], alone[k][0])
        assert res[k][1]["report"] == alone[k][1]["report"]
    assert len({s["t_admit"] for _, s in res}) == 1
