#!/usr/bin/env python3
"""Benchmark of the LiDAR bundle-adjustment hot path on one MI355X.

Default workload (the headline): 256 independent window problems with 20..400
poses and 5k..80k planar voxels each (the batched workload; seeded synthetic
raw-sum clusters, 37M clusters, 1.85G virtual points) held in one problem in
the precision form (FP32 voxel-centred clusters, FP64 eigensolve, increment
solves and pose update).  A step is one complete 10-iteration LM solve of all
windows: every iteration evaluates all voxel residuals at the trial poses, the
surrogate gradient and Hessian at accepted poses, and solves the damped
increments, all on the device, replayed from one captured graph.  The batched
FP64 form and the plain per-problem FP64 path run beside it.  The problem is
built once before the timed region; its build time is reported apart.

Other workloads: --workload window (500-pose single window built from 117M
points), city, served, scaling, pipeline.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, 8 TB/s
FP64_MFMA_PEAK_TFS = 78.6       # MI355X dense FP64 matrix
CLUSTER_BYTES = 8 + 24 + 48 + 4  # N (f64), mu (3 f64), S (6 f64), scan or slot id (i32)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_scene(workload: str):
    import scenes
    if workload == "window":
        return scenes.window_config(seed=2000)
    if workload == "tiny":
        return scenes.tiny_config(seed=1000)
    raise SystemExit(f"unknown workload {workload}")


def cpu_baseline(sc, mode_name: str, iters: int):
    """The FP64 oracle, single thread, on `iters` LM iterations of the same problem."""
    import oracle
    t0 = time.perf_counter()
    cl = oracle.scene_clusters(sc)
    t_build = time.perf_counter() - t0
    mode = oracle.MM if mode_name == "mm" else oracle.COUPLED
    t0 = time.perf_counter()
    _, rep, _ = oracle.lm(mode, cl, sc.poses_init, iters)
    dt = time.perf_counter() - t0
    return dt, rep, t_build


def _measured_traffic(key: str):
    """HBM bytes per launch of an evaluation pass on the single-window workload
    from the committed rocprofv3 byte-counter summary, or None once the kernel
    source differs from the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "window500_traffic.md")
    src = os.path.join(ROOT, "paper_2608_14266_amd", "csrc", "ba_eval.hip")
    try:
        vals = dict(line.split()[:2] for line in open(path) if line.startswith("traffic_"))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if vals.get("traffic_source_sha256") != sha or key not in vals:
        return None
    return int(float(vals[key]))


def _pose_diff_aligned(Pa, Pb):
    """Max rotation angle (rad) and translation difference (m) between two
    pose sets after removing the gauge: Pa moved by the rigid motion that maps
    its pose 0 onto Pb's pose 0."""
    import numpy as np
    Ra = Pa[:, :9].reshape(-1, 3, 3); ta = Pa[:, 9:]
    Rb = Pb[:, :9].reshape(-1, 3, 3); tb = Pb[:, 9:]
    Rg = Rb[0] @ Ra[0].T
    tg = tb[0] - Rg @ ta[0]
    Ra2 = np.einsum("ij,njk->nik", Rg, Ra)
    ta2 = ta @ Rg.T + tg
    c = (np.einsum("nij,nij->n", Ra2, Rb) - 1.0) / 2.0
    return float(np.arccos(np.clip(c, -1.0, 1.0)).max()), float(np.abs(ta2 - tb).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=20, help="LM iterations per solve")
    ap.add_argument("--mode", choices=["mm", "coupled"], default=None,
                    help="Hessian form (default: mm; coupled for --workload served)")
    ap.add_argument("--workload", choices=["window", "tiny", "city", "batch", "served", "scaling", "pipeline"],
                    default="batch",
                    help="batch: 256 uneven windows (the headline); window: 500-pose single window; city: "
                         "2000-pose 5 km precision-form map; served: Poisson request stream; scaling: "
                         "build time against points and per-iteration times against clusters and poses; "
                         "pipeline: unlabelled points -> voxelize -> build -> solve")
    ap.add_argument("--rates", type=str, default="50,200,500", help="served: request arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=120, help="served: number of requests per rate")
    ap.add_argument("--slots", type=int, default=8, help="served: concurrent requests")
    ap.add_argument("--batch", type=int, default=1,
                    help="served: queued requests a slot fuses into one problem of windows (1: one per problem)")
    ap.add_argument("--windows", type=int, default=256, help="batch: number of windows")
    ap.add_argument("--sweep-poses", type=str, default="1000,2000,5000,10000,20000",
                    help="scaling: pose counts of the city-law sweep")
    ap.add_argument("--sweep-points", type=str, default="0.25,0.5,1,2",
                    help="scaling: window-scene scale factors of the preprocessing sweep (1 = 117M points)")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle LM iterations timed for cpu_baseline (default: 50 mm, about 12 s on one core; 1 coupled)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-leg", action="store_true",
                    help="skip the FP32 precision-form run on the same workload")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch choices")
    ap.add_argument("--no-plain-leg", action="store_true",
                    help="batch: skip the plain per-problem FP64 path (for counter runs of the batched passes)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device to device three times "
                         "(a plain copy kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.mode is None:
        args.mode = "coupled" if args.workload == "served" else "mm"
    if args.cpu_iters is None:
        args.cpu_iters = 50 if args.mode == "mm" else 1
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2608_14266_amd as ba
    from paper_2608_14266_amd import build as hb

    if not os.path.exists(hb.LIB):
        log("libba not built; building")
        hb.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload in ("city", "batch", "served", "scaling", "pipeline"):
        import bench_legs
        out = {"city": bench_legs.city, "batch": bench_legs.batch, "served": bench_legs.served,
               "scaling": bench_legs.scaling, "pipeline": bench_legs.pipeline}[args.workload](args)
        print(json.dumps(out), flush=True)
        _calibration_copy(args, dev)
        return

    t0 = time.perf_counter()
    sc = make_scene(args.workload)
    log(f"scene {sc.name}: {sc.n_points} points, {sc.n_clusters} clusters, generated in "
        f"{time.perf_counter() - t0:.1f}s")
    f = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    xs, ys, zs = f(sc.x, torch.float64), f(sc.y, torch.float64), f(sc.z, torch.float64)
    scan, vox = f(sc.scan, torch.int32), f(sc.voxel, torch.int32)
    torch.cuda.synchronize()
    # build once (a0), timed apart: several repeats, best reported
    build_ms = []
    prob = None
    for _ in range(3):
        if prob is not None:
            prob.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = ba.build_clusters(xs, ys, zs, scan, vox, sc.n_scans, sc.n_voxels)
        torch.cuda.synchronize()
        build_ms.append(1e3 * (time.perf_counter() - t0))
    info = prob.info()
    V, C, N = info["n_voxels"], info["n_clusters"], info["n_scans"]
    log(f"built: {V} voxels, {C} clusters, {info['n_wave_groups']} wave groups, "
        f"{info['n_pose_chunks']} pose chunks, build {min(build_ms):.1f} ms")
    mode = ba.MODE_MM if args.mode == "mm" else ba.MODE_COUPLED
    P0 = f(sc.poses_init, torch.float64)
    P = P0.clone().contiguous()
    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuning = ba.tuned(prob, P0, cache_path=None, reps=5)
        log(f"autotuned in {time.perf_counter() - t0:.2f}s: {tuning}")

    def step():
        P.copy_(P0)
        reps, _ = ba.iterate(prob, P, mode, max_iters=args.iters, trace=False)
        return reps

    for w in range(args.warmup):
        step()
        log(f"warmup {w + 1}/{args.warmup}")
    # timed region: each solve replays the captured iteration graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = None
    for k in range(args.steps):
        reps = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel timing: the same K solves launched eagerly with HIP events around
    # every launch of the eval and factorization kernels
    ba.profile_reset()
    ba.profile_enable(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ba.profile_enable(False)
    vox_ms, vox_n = ba.profile_query("k_vox")
    pose_ms, pose_n = ba.profile_query("k_pose")
    syrk_ms, syrk_n = ba.profile_query("k_syrk")
    trsm_ms, trsm_n = ba.profile_query("k_trsm")
    potf2_ms, potf2_n = ba.profile_query("k_potf2")
    flow_ms, flow_n = ba.profile_query("k_chol_flow")
    bs_ms, bs_n = ba.profile_query("k_backsub_flow")
    ba.profile_reset()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    evals = V * args.iters * args.steps
    value = evals / elapsed
    lm_iters_s = args.iters * args.steps / elapsed
    log(f"timed {args.steps} solves: {ms_per_step:.3f} ms/solve, cost {reps[0]['cost_initial']:.6e} -> "
        f"{reps[0]['cost_final']:.6e}, accepted {reps[0]['n_accepted']}/{reps[0]['iters']}")

    # roofline of the dominant kernel (algorithmic bytes / measured launch time)
    n_groups, n_chunks = info["n_wave_groups"], info["n_pose_chunks"]
    vox_bytes = C * CLUSTER_BYTES + V * 64 + N * 96 + n_groups * 8
    pose_bytes = C * CLUSTER_BYTES + V * 56 + N * 96 + n_chunks * 27 * 8
    # k_pose launches that did work: one per accepted iteration plus the start and final ones
    pose_work = args.steps * (reps[0]["n_accepted"] + 1)
    kern = {
        "k_vox": dict(avg_us=1e3 * vox_ms / max(vox_n, 1), launches=vox_n, bytes=vox_bytes),
        "k_pose": dict(avg_us=1e3 * pose_ms / max(pose_n, 1), launches=pose_n, bytes=pose_bytes,
                       launches_with_work=pose_work),
    }
    for k, d in kern.items():
        d["gbs"] = d["bytes"] / (d["avg_us"] * 1e-6) / 1e9 if d["avg_us"] > 0 else 0.0
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    traffic = _measured_traffic(f"traffic_{dom}_f64_bytes") if args.workload == "window" else None
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(kern[dom]["gbs"], 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(kern[dom]["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": kern[dom]["bytes"], "avg_launch_us": round(kern[dom]["avg_us"], 3)}
    if args.mode == "coupled" and flow_n > 0:
        # dataflow factorization (one launch per solve, matrices up to 6144
        # rows): algorithmic flops n^3/3 of one 6N x 6N Cholesky per launch
        n = 6 * N
        fl = n ** 3 / 3
        tfs = fl * flow_n / (flow_ms * 1e-3) / 1e12
        kern["k_chol_flow"] = dict(avg_us=1e3 * flow_ms / flow_n, launches=flow_n, flops=fl)
        if bs_n > 0:
            kern["k_backsub_flow"] = dict(avg_us=1e3 * bs_ms / bs_n, launches=bs_n)
        roof = {"kernel": "k_chol_flow", "bound": "mfma", "achieved": round(tfs, 3),
                "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": round(tfs / FP64_MFMA_PEAK_TFS, 4),
                "traffic": None, "flops_per_factorization": fl, "avg_launch_us": round(1e3 * flow_ms / flow_n, 3)}
    elif args.mode == "coupled" and syrk_n > 0:
        # dense factorization on FP64 matrix cores: algorithmic flops of the
        # panel solves (rows below x 64 x 64 x 2) and trailing updates
        # (rows below^2 x 64, lower half) of one 6N x 6N factorization
        n = 6 * N
        fl_trsm = fl_syrk = 0
        for st in range((n + 63) // 64):
            below = n - 64 * (st + 1)
            if below > 0:
                fl_trsm += below * 64 * 64 * 2
                fl_syrk += below * below * 64
        n_fact = potf2_n / ((n + 63) // 64)   # one diagonal-block factor per 64-wide step
        tfs = (fl_trsm + fl_syrk) * n_fact / ((syrk_ms + trsm_ms) * 1e-3) / 1e12
        kern["k_syrk"] = dict(avg_us=1e3 * syrk_ms / max(syrk_n, 1), launches=syrk_n)
        kern["k_trsm"] = dict(avg_us=1e3 * trsm_ms / max(trsm_n, 1), launches=trsm_n)
        kern["k_potf2"] = dict(avg_us=1e3 * potf2_ms / max(potf2_n, 1), launches=potf2_n)
        kern["factorization"] = dict(count=n_fact, flops=fl_trsm + fl_syrk)
        roof = {"kernel": "k_syrk+k_trsm", "bound": "mfma", "achieved": round(tfs, 3),
                "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": round(tfs / FP64_MFMA_PEAK_TFS, 4),
                "traffic": None, "flops_per_factorization": fl_trsm + fl_syrk,
                "avg_launch_us": round(1e3 * syrk_ms / max(syrk_n, 1), 3)}

    # precision form on the same workload: FP32 voxel-centred clusters, same
    # LM, same number of solves; final poses compared with the FP64 run
    prec = None
    if not args.no_precision_leg:
        P64_final = P.clone()
        prob32 = ba.build_clusters(xs, ys, zs, scan, vox, sc.n_scans, sc.n_voxels, precision=ba.PREC_F32,
                                   ref_poses=P0)
        tuning32 = None if args.no_autotune else ba.tuned(prob32, P0, cache_path=None, reps=5)
        P32 = P0.clone().contiguous()

        def step32():
            P32.copy_(P0)
            return ba.iterate(prob32, P32, mode, max_iters=args.iters, trace=False)[0]

        for _ in range(args.warmup):
            step32()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for _ in range(args.steps):
            reps32 = step32()
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        ba.profile_reset()
        ba.profile_enable(True)
        step32()
        torch.cuda.synchronize()
        ba.profile_enable(False)
        v32_ms, v32_n = ba.profile_query("k_vox")
        p32_ms, p32_n = ba.profile_query("k_pose")
        ba.profile_reset()
        inf32 = prob32.info()
        vox32_bytes = C * inf32["cluster_bytes"] + V * (64 + 32) + N * 2 * 96 + n_groups * 8
        vox32_us = 1e3 * v32_ms / max(v32_n, 1)
        ang, dt = _pose_diff_aligned(P32.cpu().numpy(), P64_final.cpu().numpy())
        prec = {"value": V * args.iters * args.steps / (t5 - t4),
                "ms_per_step": 1e3 * (t5 - t4) / args.steps,
                "cluster_bytes": inf32["cluster_bytes"], "device_bytes": inf32["device_bytes"],
                "k_vox_avg_us": round(vox32_us, 3), "k_pose_avg_us": round(1e3 * p32_ms / max(p32_n, 1), 3),
                "k_vox_gbs": round(vox32_bytes / (vox32_us * 1e-6) / 1e9, 2) if vox32_us > 0 else 0.0,
                "final_cost": reps32[0]["cost_final"], "tuning": tuning32,
                "final_cost_rel_diff_vs_f64": abs(reps32[0]["cost_final"] - reps[0]["cost_final"])
                / reps[0]["cost_final"],
                "pose_diff_vs_f64_gauge_aligned": {"rad": ang, "m": dt}}
        log(f"precision form: {prec['ms_per_step']:.3f} ms/solve, k_vox {vox32_us:.2f} us, "
            f"pose diff {ang:.2e} rad {dt:.2e} m")
        prob32.close()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_iters} LM iterations")
        dt, rep, tb = cpu_baseline(sc, args.mode, args.cpu_iters)
        cpu = {"value": V * args.cpu_iters / dt, "unit": "plane-voxel evals/s", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_iters} LM iterations ({args.mode}) of the full {sc.name} problem, "
                         f"single thread, FP64; cluster build ({tb:.1f}s) untimed",
               "seconds": round(dt, 3)}
        log(f"cpu baseline {cpu['value']:.4g} evals/s ({dt:.2f}s)")

    out = {
        "metric": "plane-voxel evals/s",
        "value": value,
        "unit": "plane-voxel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{sc.name} ({args.mode}, {args.iters} LM iterations per step)",
                   "poses": N, "voxels": V, "clusters": C, "points": sc.n_points, "lm_iters": args.iters,
                   "mode": args.mode},
        "lm_iters_per_s": lm_iters_s,
        "ms_per_step_eager_profiled": round(1e3 * (t3 - t2) / args.steps, 4),
        "build_ms": round(min(build_ms), 3),
        "tuning": tuning,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in d.items()}
                    for k, d in kern.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "final_cost": reps[0]["cost_final"],
        "precision_form": prec,
    }
    print(json.dumps(out), flush=True)
    _calibration_copy(args, dev)


def _calibration_copy(args, dev):
    """A plain device-to-device copy of known size (three times), after the
    measured work: the reference that scales hardware byte counters."""
    if args.calib_copy_mib <= 0:
        return
    import torch
    nb = args.calib_copy_mib << 20
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy: 3 x {args.calib_copy_mib} MiB")


if __name__ == "__main__":
    main()
