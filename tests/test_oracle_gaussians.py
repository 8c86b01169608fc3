"""Pins of the oracle's triangle frame and Gaussian re-pose (CPU only).

The paper gives no binding formula (Sec. 3.2), so the reading is pinned by a
hand-worked example, closed-form invariants and independent library routines
(scipy's rotation conversions), never by re-typing the oracle's formulas.
"""

import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import gaussians as og

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_tris(rng, n):
    v = rng.normal(size=(3, n, 3))
    return v[0], v[1], v[2]


def _rand_binding(rng, nf, g):
    q = rng.normal(size=(4, g))
    q /= np.linalg.norm(q, axis=0)
    r1, r2 = rng.random(g), rng.random(g)
    s = np.sqrt(r1)
    return {"face": rng.integers(0, nf, g), "bary": np.stack([s * (1 - r2), s * r2]),
            "q_local": q, "log_scale": rng.normal(-1.0, 0.5, size=(3, g))}


def test_worked_example():
    gold = json.load(open(os.path.join(GOLD, "frame_worked.json")))
    v = np.array(gold["verts"], dtype=np.float64)
    R, nh, deg = og.triangle_frame(v[0:1], v[1:2], v[2:3])
    assert not deg[0]
    np.testing.assert_array_equal(R[0], np.array(gold["R_f"], dtype=np.float64))
    np.testing.assert_array_equal(nh[0], gold["normal"])
    verts = v.T.copy()
    faces = np.array([[0], [1], [2]])
    b = {"face": np.array([0]), "bary": np.array([[gold["bary"][0]], [gold["bary"][1]]]),
         "q_local": np.array([[1.0], [0.0], [0.0], [0.0]]),
         "log_scale": np.array(gold["log_scale"], dtype=np.float64)[:, None]}
    out = og.repose(verts, faces, b)
    np.testing.assert_allclose(out["quat"][:, 0], gold["quat"], atol=1e-15)
    np.testing.assert_allclose(out["cov"][:, 0], gold["cov_packed"], atol=1e-13)
    np.testing.assert_allclose(out["mean"][:, 0], gold["mean"], atol=1e-15)
    out = og.repose(verts, faces, b, offset=np.array([gold["offset"]]))
    np.testing.assert_allclose(out["mean"][:, 0], gold["mean_offset"], atol=1e-15)


def test_identity_frame_exact():
    v0, v1, v2 = np.array([[0.0, 0, 0]]), np.array([[1.0, 0, 0]]), np.array([[0.0, 1, 0]])
    R, nh, deg = og.triangle_frame(v0, v1, v2)
    np.testing.assert_array_equal(R[0], np.eye(3))
    np.testing.assert_array_equal(nh[0], [0, 0, 1])


def test_frame_orthonormal_right_handed():
    rng = np.random.default_rng(1)
    v0, v1, v2 = _rand_tris(rng, 500)
    R, nh, deg = og.triangle_frame(v0, v1, v2)
    assert not deg.any()
    np.testing.assert_allclose(np.transpose(R, (0, 2, 1)) @ R, np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # normal perpendicular to both edges, tangent along the first edge
    np.testing.assert_allclose((nh * (v1 - v0)).sum(1), 0, atol=1e-12)
    np.testing.assert_allclose((nh * (v2 - v0)).sum(1), 0, atol=1e-12)
    e1 = (v1 - v0) / np.linalg.norm(v1 - v0, axis=1, keepdims=True)
    np.testing.assert_allclose(R[:, :, 0], e1, atol=1e-12)
    # the normal follows the winding: positive orientation of (e1, e2, n)
    assert (np.linalg.det(np.stack([v1 - v0, v2 - v0, nh], 1)) > 0).all()


def test_degenerate_face():
    v = np.array([[0.0, 0, 0]])
    R, nh, deg = og.triangle_frame(v, v, np.array([[1.0, 0, 0]]))
    assert deg[0]
    np.testing.assert_array_equal(R[0], np.eye(3))
    np.testing.assert_array_equal(nh[0], 0)


def test_quaternion_matrix_against_scipy():
    rng = np.random.default_rng(2)
    q = rng.normal(size=(400, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = og.quat_to_matrix(q)
    Rs = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()          # scipy is scalar-last
    np.testing.assert_allclose(R, Rs, atol=1e-14)
    qs = Rotation.from_matrix(Rs).as_quat()[:, [3, 0, 1, 2]]
    qo = og.matrix_to_quat(Rs)
    sign = np.sign((qs * qo).sum(1))
    np.testing.assert_allclose(qo, qs * sign[:, None], atol=1e-13)
    assert (qo[:, 0] >= 0).all()


def test_shepperd_all_branches_and_sign_rule():
    # 180-degree turns hit the R00 / R11 / R22 branches with w == 0
    for axis in np.eye(3):
        R = Rotation.from_rotvec(np.pi * axis).as_matrix()[None]
        q = og.matrix_to_quat(R)[0]
        assert q[0] == pytest.approx(0.0, abs=1e-15)
        np.testing.assert_allclose(q[1:], axis, atol=1e-15)
    q = og.canonical_sign(np.array([[0.0, 0.0, -1.0, 0.5], [-0.2, 0.1, 0.0, 0.0], [0.0, -0.0, 0.0, -1.0]]))
    assert q[0, 2] > 0 and q[1, 0] > 0 and q[2, 3] > 0


@pytest.mark.parametrize("seed", [3, 4])
def test_rigid_motion_equivariance(seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(3, 60))
    F = rng.integers(0, 60, size=(3, 80))
    F = F[:, (F[0] != F[1]) & (F[1] != F[2]) & (F[0] != F[2])]
    b = _rand_binding(rng, F.shape[1], 300)
    off = rng.normal(0, 0.1, 300)
    Q = Rotation.random(random_state=seed).as_matrix()
    T = rng.normal(size=(3, 1))
    base = og.repose(V, F, b, offset=off)
    moved = og.repose(Q @ V + T, F, b, offset=off)
    np.testing.assert_allclose(moved["mean"], Q @ base["mean"] + T, atol=1e-12)
    np.testing.assert_allclose(moved["rot"], Q[None] @ base["rot"], atol=1e-12)
    S0 = og.unpack_sym(base["cov"])
    S1 = og.unpack_sym(moved["cov"])
    np.testing.assert_allclose(S1, Q[None] @ S0 @ Q.T[None], atol=1e-12)
    # quaternion composes with the motion's quaternion (up to sign)
    qQ = Rotation.from_matrix(Q).as_quat()[[3, 0, 1, 2]]
    qb = base["quat"].T
    w1, x1, y1, z1 = qQ
    w2, x2, y2, z2 = qb.T
    comp = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    d = np.minimum(np.linalg.norm(comp - moved["quat"].T, axis=1), np.linalg.norm(comp + moved["quat"].T, axis=1))
    assert d.max() < 1e-12


def test_covariance_spectrum():
    rng = np.random.default_rng(5)
    V = rng.normal(size=(3, 30))
    F = np.stack([np.arange(0, 30, 3), np.arange(1, 30, 3), np.arange(2, 30, 3)])
    b = _rand_binding(rng, 10, 200)
    out = og.repose(V, F, b)
    S = og.unpack_sym(out["cov"])
    ev = np.sort(np.linalg.eigvalsh(S), axis=1)
    s2 = np.sort(np.exp(2 * b["log_scale"]).T, axis=1)
    np.testing.assert_allclose(ev, s2, rtol=1e-10)


def test_barycentric_corners_are_vertices():
    rng = np.random.default_rng(6)
    V = rng.normal(size=(3, 3))
    F = np.array([[0], [1], [2]])
    for k, bary in enumerate([(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]):
        b = {"face": np.array([0]), "bary": np.array(bary)[:, None], "q_local": np.array([[1.0], [0], [0], [0]]),
             "log_scale": np.zeros((3, 1))}
        out = og.repose(V, F, b)
        np.testing.assert_array_equal(out["mean"][:, 0], V[:, k])


def test_rest_pose_round_trip():
    rng = np.random.default_rng(7)
    from synth import uv_sphere
    xhat, f = uv_sphere(12, 6)
    V = xhat.T * (1 + 0.1 * rng.random(xhat.shape[0]))
    F = f.T
    g = 400
    fid = rng.integers(0, F.shape[1], g)
    # world-space rest Gaussians: points on or near their faces, random rotations
    tri = F[:, fid]
    r1, r2 = rng.random(g), rng.random(g)
    s = np.sqrt(r1)
    w = np.stack([1 - s, s * (1 - r2), s * r2])
    mean0 = sum(w[k] * V[:, tri[k]] for k in range(3))
    _, nh, _ = og.triangle_frame(V[:, tri[0]].T, V[:, tri[1]].T, V[:, tri[2]].T)
    mean0 = mean0 + 0.01 * rng.normal(size=g) * nh.T
    quat0 = Rotation.random(g, random_state=8).as_quat()[:, [3, 0, 1, 2]].T
    ls = rng.normal(-3, 0.3, size=(3, g))
    binding, delta = og.bind_rest_pose(V, F, fid, mean0, quat0, ls)
    out = og.repose(V, F, binding, offset=delta)
    np.testing.assert_allclose(out["mean"], mean0, atol=1e-13)
    q0 = og.canonical_sign(quat0.T)
    d = np.minimum(np.linalg.norm(out["quat"].T - q0, axis=1), np.linalg.norm(out["quat"].T + q0, axis=1))
    assert d.max() < 1e-13
