"""The CPU oracle built with gcc's address and undefined-behaviour sanitizers
(host code only, no GPU) and run through every entry point on two small
scenes: no sanitizer report, and the same values as the uninstrumented
oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("san") / "orc_san")
    cmd = [gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-std=gnu11", os.path.join(ORC, "ba_oracle.c"),
           os.path.join(ORC, "sanitize_driver.c"), "-o", out, "-lm", "-lquadmath"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _write_scene(path, sc):
    with open(path, "wb") as f:
        np.array([sc.x.shape[0]], np.int64).tofile(f)
        np.array([sc.n_scans, sc.n_voxels], np.int32).tofile(f)
        for a in (sc.x, sc.y, sc.z):
            np.ascontiguousarray(a, np.float64).tofile(f)
        for a in (sc.scan, sc.voxel):
            np.ascontiguousarray(a, np.int32).tofile(f)
        np.ascontiguousarray(sc.poses_init, np.float64).tofile(f)


@pytest.mark.parametrize("name", ["tiny", "edge"])
def test_oracle_under_sanitizers(driver, orc, tmp_path, name):
    if name == "tiny":
        sc = scenes.tiny_config(seed=1000)
    else:
        # single-scan voxels, one-point clusters, an unobserved scan
        sc = scenes.small_scene(seed=77, n_scans=6, n_planes=20, m_range=(1, 3), pts_per_obs=(1, 12),
                                path_len=8.0, offset_range=8.0)
    path = str(tmp_path / "scene.bin")
    _write_scene(path, sc)
    # the environment is passed on unchanged apart from the sanitizer options
    # (a preloaded library of the host stays preloaded: ASan then skips its
    # link-order check)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    vals = {}
    for line in r.stdout.splitlines():
        w = line.split()
        if w[0] == "stats":
            vals["cost"] = float(w[3])
        elif w[0] == "lm":
            vals[f"lm{w[2][0]}"] = float(w[6])
    cl = orc.scene_clusters(sc)
    assert vals["cost"] == orc.cost(cl, sc.poses_init)
    _, _, c_mm = orc.lm(orc.MM, cl, sc.poses_init, 12, tol_g=1e-9, max_rejects=10)
    _, _, c_cp = orc.lm(orc.COUPLED, cl, sc.poses_init, 12, tol_g=1e-9, max_rejects=10, exact_below=0.1)
    assert vals["lm0"] == c_mm and vals["lm1"] == c_cp
