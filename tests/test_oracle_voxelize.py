"""Pins of the voxelization oracle (Sec. IV-A, Eq. 4-5, Alg. 1) against
references independent of its sort-and-reduce formulation: grouping by a
dictionary on small inputs, the exact identity between level k at edge d and
level 1 at edge 2^(k-1) d, a box whose covariance is known in closed form, and
count conservation."""
import math

import numpy as np
import pytest

from oracle import voxelize as vz


def _poses(rng, n):
    P = np.zeros((n, 12))
    for j in range(n):
        a = rng.uniform(-np.pi, np.pi)
        c, s = math.cos(a), math.sin(a)
        P[j, :9] = [c, -s, 0, s, c, 0, 0, 0, 1]
        P[j, 9:] = rng.uniform(-5, 5, 3)
    return P


def _cloud(seed, n=300, n_scans=3):
    rng = np.random.default_rng(seed)
    x, y, z = rng.uniform(-4, 4, (3, n))
    scan = rng.integers(0, n_scans, n)
    return x, y, z, scan, _poses(rng, n_scans)


def test_levels_match_dictionary_grouping():
    """Every level's clusters equal a dictionary grouping of the points by
    (floor(w / d) halved k-1 times, scan): same keys in sorted order, counts,
    and sums of p and p p^T."""
    x, y, z, scan, P = _cloud(1)
    d, L = 0.9, 3
    res = vz.voxelize(x, y, z, scan, P, d, L, tau=0.3)
    for k in range(1, L + 1):
        groups = {}
        for i in range(x.shape[0]):
            R = P[scan[i], :9].reshape(3, 3)
            w = R @ np.array([x[i], y[i], z[i]]) + P[scan[i], 9:]
            key = tuple(math.floor(math.floor(w[r] / d) / 2 ** (k - 1)) for r in range(3)) + (int(scan[i]),)
            g = groups.setdefault(key, [0, np.zeros(3), np.zeros((3, 3))])
            p = np.array([x[i], y[i], z[i]])
            g[0] += 1
            g[1] += p
            g[2] += np.outer(p, p)
        keys = sorted(groups)
        cl = res["levels"][k - 1]
        got = [tuple(int(v) for v in c) + (int(s),) for c, s in zip(cl["cell"], cl["scan"])]
        assert got == keys
        for q, key in enumerate(keys):
            n, s1, s2 = groups[key]
            assert cl["count"][q] == n
            assert np.allclose(cl["sum"][q], s1, rtol=1e-13, atol=1e-13)
            iu = [s2[0, 0], s2[0, 1], s2[0, 2], s2[1, 1], s2[1, 2], s2[2, 2]]
            assert np.allclose(cl["sumsq"][q], iu, rtol=1e-13, atol=1e-12)


def test_level_k_equals_level_one_at_scaled_edge():
    """floor(floor(w/d) / 2^(k-1)) = floor(w / (2^(k-1) d)) holds exactly in
    binary floating point (scaling by a power of two commutes with rounding),
    so level k at edge d and level 1 at edge 2^(k-1) d form the same clusters."""
    x, y, z, scan, P = _cloud(2, n=3000, n_scans=5)
    d = 0.37
    a = vz.voxelize(x, y, z, scan, P, d, 3, tau=0.3)["levels"]
    for k in (2, 3):
        b = vz.voxelize(x, y, z, scan, P, d * 2 ** (k - 1), 1, tau=0.3)["levels"][0]
        assert np.array_equal(a[k - 1]["cell"], b["cell"])
        assert np.array_equal(a[k - 1]["scan"], b["scan"])
        assert np.array_equal(a[k - 1]["count"], b["count"])
        assert np.allclose(a[k - 1]["sum"], b["sum"], rtol=1e-12, atol=1e-12)
        assert np.allclose(a[k - 1]["lam"], b["lam"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("above", [True, False])
def test_box_corners_select_by_closed_form_ratio(above):
    """The 8 corners of a box with half-extents (a, b, h), h < b < a, have
    covariance diag(a^2, b^2, h^2): the cell is kept exactly when
    tau > h^2 / b^2."""
    a_, b_, h = 0.3, 0.2, 0.05
    corners = np.array([[sx * a_, sy * b_, sz * h] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)])
    c = np.array([10.5, -3.5, 2.5])          # centre of the level-1 cell [10, 11) x [-4, -3) x [2, 3) at d = 1
    pts = corners + c
    P = np.array([[1.0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]])
    ratio = h * h / (b_ * b_)
    tau = ratio * (1.001 if above else 0.999)
    res = vz.voxelize(pts[:, 0], pts[:, 1], pts[:, 2], np.zeros(8, np.int64), P, 1.0, 2, tau=tau)
    for lvl in res["levels"]:
        assert lvl["n_voxels"] == 1
        assert np.allclose(lvl["lam"][0], [h * h, b_ * b_, a_ * a_], rtol=1e-12)
        assert bool(lvl["keep"][0]) == above
    assert res["out"]["n_voxels"] == (2 if above else 0)


def test_counts_are_conserved_and_cells_nest():
    x, y, z, scan, P = _cloud(3, n=5000, n_scans=7)
    res = vz.voxelize(x, y, z, scan, P, 0.5, 4, tau=0.2, min_scans=2)
    for k, lvl in enumerate(res["levels"]):
        assert lvl["count"].sum() == x.shape[0]
        if k:
            # every cluster's cell is the parent of some finer cluster's cell with the same scan
            fine = {(tuple(c >> 1), s) for c, s in zip(res["levels"][k - 1]["cell"], res["levels"][k - 1]["scan"])}
            assert {(tuple(c), s) for c, s in zip(lvl["cell"], lvl["scan"])} == fine
        assert np.all(lvl["n_scans"][lvl["keep"]] >= 2)
    out = res["out"]
    assert out["count"].sum() == sum(int(l["count"][np.repeat(l["keep"], l["n_scans"])].sum())
                                     for l in res["levels"])


def test_plane_is_kept_and_blob_rejected():
    """Points on a tilted plane (1 mm noise) form planar cells; an isotropic
    blob does not."""
    rng = np.random.default_rng(4)
    n = 4000
    u, v = rng.uniform(0, 2, (2, n))
    nrm = np.array([0.3, -0.2, 0.93])
    nrm /= np.linalg.norm(nrm)
    e1 = np.cross(nrm, [1.0, 0, 0]); e1 /= np.linalg.norm(e1)
    e2 = np.cross(nrm, e1)
    plane = u[:, None] * e1 + v[:, None] * e2 + rng.normal(0, 1e-3, n)[:, None] * nrm
    blob = rng.normal(0, 0.3, (n, 3)) + 20.0
    pts = np.concatenate([plane, blob])
    P = np.array([[1.0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]])
    res = vz.voxelize(pts[:, 0], pts[:, 1], pts[:, 2], np.zeros(2 * n, np.int64), P, 0.5, 2, tau=0.01)
    for lvl in res["levels"]:
        plane_cells = (lvl["cell"][lvl["vstart"]] < 10).all(axis=1)
        dense = np.add.reduceat(lvl["count"], lvl["vstart"]) >= 50
        assert np.all(lvl["keep"][plane_cells & dense])
        assert not np.any(lvl["keep"][~plane_cells & dense])


def test_cells_of_fewer_than_three_points_or_a_line_are_not_planes():
    """One or two points, or points on a line, span no plane (their l1 is
    rounding); three points in general position always lie in a plane."""
    P = np.array([[1.0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]])
    cases = {  # cell centre offsets inside [0, 1)^3 cells at d = 1
        "one": [[0.5, 0.5, 0.5]],
        "two": [[0.2, 0.3, 0.4], [0.7, 0.6, 0.5]],
        "line": [[0.1, 0.1, 0.1], [0.4, 0.4, 0.4], [0.9, 0.9, 0.9]],
        "three": [[0.1, 0.2, 0.3], [0.8, 0.2, 0.5], [0.4, 0.9, 0.1]],
    }
    for name, pts in cases.items():
        p = np.asarray(pts) + np.array([3.0, -2.0, 7.0])
        res = vz.voxelize(p[:, 0], p[:, 1], p[:, 2], np.zeros(len(p), np.int64), P, 1.0, 1, tau=0.5)
        assert bool(res["levels"][0]["keep"][0]) == (name == "three"), name
