"""ctypes binding of the plain FP64 CPU oracle (``ba_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg are the only callers.  The GPU product path
never imports this package.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ba_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MM, COUPLED, EXACT = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build(force=True)
    lib = ct.CDLL(LIB)
    P = ct.c_void_p
    i64, i32, dbl, cint = ct.c_int64, ct.c_int32, ct.c_double, ct.c_int
    lib.orc_points_to_clusters.restype = i64
    lib.orc_points_to_clusters.argtypes = [i64, P, P, P, P, P, P, P, P, P, P]
    lib.orc_points_to_raw_sums.restype = i64
    lib.orc_points_to_raw_sums.argtypes = [i64, P, P, P, P, P, P, P, P, P, P]
    lib.orc_center_raw_sums.restype = None
    lib.orc_center_raw_sums.argtypes = [i64, P, P, P, P, P]
    lib.orc_eig3.restype = None
    lib.orc_eig3.argtypes = [P, P, P]
    lib.orc_voxel_stats.restype = cint
    lib.orc_voxel_stats.argtypes = [i64, P, P, P, P, P, i32, i32, P, P, P, P, P, P]
    lib.orc_cost.restype = dbl
    lib.orc_cost.argtypes = [i64, P, P, P, P, P, i32, i32, P]
    lib.orc_majorizer.restype = dbl
    lib.orc_majorizer.argtypes = [cint, i64, P, P, P, P, P, i32, i32, P, P]
    lib.orc_eval.restype = cint
    lib.orc_eval.argtypes = [cint, i64, P, P, P, P, P, i32, i32, P, P, P, P, P]
    lib.orc_eval_abs.restype = cint
    lib.orc_eval_abs.argtypes = [cint, i64, P, P, P, P, P, i32, i32, P, P, P, P, P, P]
    lib.orc_solve.restype = cint
    lib.orc_solve.argtypes = [cint, i32, P, P, dbl, P]
    lib.orc_so3_exp.restype = None
    lib.orc_so3_exp.argtypes = [P, P]
    lib.orc_apply_increment.restype = None
    lib.orc_apply_increment.argtypes = [i32, P, P, P]
    lib.orc_lm.restype = cint
    lib.orc_lm.argtypes = [cint, i64, P, P, P, P, P, i32, i32, P, cint, dbl, dbl, dbl, cint, dbl, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Clusters:
    """Centred point clusters sorted by (voxel, scan)."""
    vox: np.ndarray   # (C,) int32
    scan: np.ndarray  # (C,) int32
    n: np.ndarray     # (C,) int64
    mu: np.ndarray    # (C, 3) float64
    S: np.ndarray     # (C, 6) float64  [xx xy xz yy yz zz]
    n_voxels: int
    n_scans: int

    @property
    def C(self) -> int:
        return int(self.vox.shape[0])

    def args(self):
        return (self.C, _p(self.vox), _p(self.scan), _p(self.n), _p(self.mu), _p(self.S),
                self.n_voxels, self.n_scans)


def points_to_clusters(x, y, z, scan, voxel, n_voxels, n_scans) -> Clusters:
    lib = _load()
    x, y, z = _c(x, np.float64), _c(y, np.float64), _c(z, np.float64)
    scan, voxel = _c(scan, np.int32), _c(voxel, np.int32)
    n = x.shape[0]
    cap = max(n, 1)
    cv = np.empty(cap, np.int32); cs = np.empty(cap, np.int32); cn = np.empty(cap, np.int64)
    mu = np.empty((cap, 3)); S = np.empty((cap, 6))
    C = lib.orc_points_to_clusters(n, _p(x), _p(y), _p(z), _p(scan), _p(voxel), _p(cv), _p(cs), _p(cn),
                                   _p(mu), _p(S))
    if C < 0:
        raise MemoryError("oracle: allocation failed")
    return Clusters(cv[:C].copy(), cs[:C].copy(), cn[:C].copy(), mu[:C].copy(), S[:C].copy(),
                    int(n_voxels), int(n_scans))


def scene_clusters(scene) -> Clusters:
    return points_to_clusters(scene.x, scene.y, scene.z, scene.scan, scene.voxel, scene.n_voxels,
                              scene.n_scans)


def points_to_raw_sums(x, y, z, scan, voxel):
    """(vox, scan, n, sum p (C,3), sum p p^T (C,6)) sorted by (voxel, scan)."""
    lib = _load()
    x, y, z = _c(x, np.float64), _c(y, np.float64), _c(z, np.float64)
    scan, voxel = _c(scan, np.int32), _c(voxel, np.int32)
    n = x.shape[0]
    cap = max(n, 1)
    cv = np.empty(cap, np.int32); cs = np.empty(cap, np.int32); cn = np.empty(cap, np.int64)
    s1 = np.empty((cap, 3)); s2 = np.empty((cap, 6))
    C = lib.orc_points_to_raw_sums(n, _p(x), _p(y), _p(z), _p(scan), _p(voxel), _p(cv), _p(cs), _p(cn),
                                   _p(s1), _p(s2))
    return cv[:C].copy(), cs[:C].copy(), cn[:C].copy(), s1[:C].copy(), s2[:C].copy()


def center_raw_sums(n, s1, s2):
    lib = _load()
    n = _c(n, np.int64); s1 = _c(s1, np.float64); s2 = _c(s2, np.float64)
    C = n.shape[0]
    mu = np.empty((C, 3)); S = np.empty((C, 6))
    lib.orc_center_raw_sums(C, _p(n), _p(s1), _p(s2), _p(mu), _p(S))
    return mu, S


def eig3(sym6):
    lib = _load()
    a = _c(sym6, np.float64)
    lam = np.empty(3); U = np.empty(9)
    lib.orc_eig3(_p(a), _p(lam), _p(U))
    return lam, U.reshape(3, 3)


def voxel_stats(cl: Clusters, poses):
    lib = _load()
    poses = _c(poses, np.float64)
    V = cl.n_voxels
    N = np.empty(V); mb = np.empty((V, 3)); A = np.empty((V, 6)); lam = np.empty((V, 3)); U = np.empty((V, 9))
    rc = lib.orc_voxel_stats(*cl.args(), _p(poses), _p(N), _p(mb), _p(A), _p(lam), _p(U))
    if rc:
        raise ValueError(f"oracle: invalid clusters ({rc})")
    return dict(N=N, mbar=mb, A=A, lam=lam, U=U.reshape(V, 3, 3))


def cost(cl: Clusters, poses) -> float:
    lib = _load()
    poses = _c(poses, np.float64)
    return float(lib.orc_cost(*cl.args(), _p(poses)))


def majorizer(kind: int, cl: Clusters, poses, poses_l) -> float:
    lib = _load()
    poses = _c(poses, np.float64); poses_l = _c(poses_l, np.float64)
    return float(lib.orc_majorizer(kind, *cl.args(), _p(poses), _p(poses_l)))


def evaluate(mode: int, cl: Clusters, poses):
    """Returns (cost, grad (6N,), hess ((N,6,6) for MM, (6N,6N) otherwise), n_degenerate)."""
    lib = _load()
    poses = _c(poses, np.float64)
    Np = cl.n_scans
    g = np.empty(6 * Np)
    H = np.empty((Np, 6, 6)) if mode == MM else np.empty((6 * Np, 6 * Np))
    c = ct.c_double(0.0)
    nd = ct.c_int64(0)
    rc = lib.orc_eval(mode, *cl.args(), _p(poses), ct.byref(c), _p(g), _p(H), ct.byref(nd))
    if rc:
        raise ValueError(f"oracle: invalid clusters ({rc})")
    return c.value, g, H, nd.value


def evaluate_abs(mode: int, cl: Clusters, poses):
    """evaluate() plus the per-entry sums of absolute contributions.  Returns
    (cost, grad, hess, grad_abs, hess_abs); the last two have the layouts of
    grad and hess and give the rounding scale of every pose block."""
    lib = _load()
    poses = _c(poses, np.float64)
    Np = cl.n_scans
    g = np.empty(6 * Np)
    ga = np.empty(6 * Np)
    shape = (Np, 6, 6) if mode == MM else (6 * Np, 6 * Np)
    H = np.empty(shape)
    Ha = np.empty(shape)
    c = ct.c_double(0.0)
    rc = lib.orc_eval_abs(mode, *cl.args(), _p(poses), ct.byref(c), _p(g), _p(H), _p(ga), _p(Ha))
    if rc:
        raise ValueError(f"oracle: invalid clusters ({rc})")
    return c.value, g, H, ga, Ha


def solve(mode: int, n_poses: int, hess, grad, mu: float):
    lib = _load()
    hess = _c(hess, np.float64); grad = _c(grad, np.float64)
    dx = np.empty(6 * n_poses)
    info = lib.orc_solve(mode, n_poses, _p(hess), _p(grad), float(mu), _p(dx))
    return dx, int(info)


def so3_exp(phi):
    lib = _load()
    phi = _c(phi, np.float64)
    R = np.empty(9)
    lib.orc_so3_exp(_p(phi), _p(R))
    return R.reshape(3, 3)


def apply_increment(poses, dx):
    lib = _load()
    poses = _c(poses, np.float64); dx = _c(dx, np.float64)
    Np = poses.shape[0]
    out = np.empty_like(poses)
    lib.orc_apply_increment(Np, _p(poses), _p(dx), _p(out))
    return out


def lm(mode: int, cl: Clusters, poses, max_iters: int, mu0: float = 1e-2, nu0: float = 2.0, tol_g: float = 0.0,
       max_rejects: int = 0, exact_below: float = 0.0):
    """Returns (final poses, report (iters, 8), final cost)."""
    lib = _load()
    P = _c(poses, np.float64).copy()
    rep = np.zeros((max(max_iters, 1), 8))
    cf = ct.c_double(0.0)
    it = lib.orc_lm(mode, *cl.args(), _p(P), int(max_iters), float(mu0), float(nu0), float(tol_g),
                    int(max_rejects), float(exact_below), _p(rep), ct.byref(cf))
    return P, rep[:it].copy(), cf.value
