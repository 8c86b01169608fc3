"""Pins of the index signed-distance grid oracle (the SDF of Sec. 3.4)."""

import numpy as np

from oracle import sdf as osdf
from oracle import closest as oc
from oracle import knn as ok
from synth.meshes import icosphere


def _sphere(level=3):
    v, f = icosphere(level)
    return v.T.astype(np.float64), f.T


def test_grid_points_layout():
    P = osdf.grid_points((1.0, -2.0, 0.5), 0.25, (3, 2, 4))
    assert P.shape == (3, 24)
    np.testing.assert_array_equal(P[:, 0], [1.0, -2.0, 0.5])
    np.testing.assert_array_equal(P[:, 1], [1.25, -2.0, 0.5])        # x fastest
    np.testing.assert_array_equal(P[:, 3], [1.0, -1.75, 0.5])
    np.testing.assert_array_equal(P[:, 6], [1.0, -2.0, 0.75])
    np.testing.assert_array_equal(P[:, 23], [1.5, -1.75, 1.25])


def test_all_faces_give_the_exact_unsigned_distance_and_sphere_signs():
    V, F = _sphere(2)
    P = osdf.grid_points((-1.5, -1.5, -1.5), 0.375, (9, 9, 9))
    allf = np.repeat(np.arange(F.shape[1])[:, None], P.shape[1], axis=1)
    r = osdf.sdf_from_faces(V, F, P, allf)
    c = oc.closest_point_mesh(V, F, P)
    np.testing.assert_allclose(np.abs(r["sdf"]), np.sqrt(c["dist2"]), rtol=1e-12, atol=1e-14)
    rad = np.linalg.norm(P, axis=0)
    # the inscribed polyhedron lies within [0.99, 1] of the centre for level 2 (chord sagitta)
    assert (r["sdf"][rad < 0.95] < 0).all() and (r["sdf"][rad > 1.05] > 0).all()
    np.testing.assert_allclose(r["sdf"][rad < 0.95], rad[rad < 0.95] - 1, atol=0.02)


def test_nearest_faces_give_the_exact_sdf_on_the_template():
    # storing each node's nearest template faces reproduces the exact SDF on the template itself
    V, F = _sphere(2)
    P = osdf.grid_points((-1.4, -1.4, -1.4), 0.4, (8, 8, 8))
    face_k, _ = ok.knn_faces(V, F, P, 1)
    allf = np.repeat(np.arange(F.shape[1])[:, None], P.shape[1], axis=1)
    a = osdf.sdf_from_faces(V, F, P, face_k)
    b = osdf.sdf_from_faces(V, F, P, allf)
    np.testing.assert_allclose(a["sdf"], b["sdf"], rtol=1e-12, atol=1e-14)


def test_trilinear_sampling_is_exact_for_linear_fields():
    lo, h, dims = (-1.0, 0.0, 2.0), 0.5, (5, 4, 3)
    P = osdf.grid_points(lo, h, dims)
    a = np.array([0.3, -1.25, 2.0])
    G = a @ P + 0.75
    rng = np.random.default_rng(0)
    Q = np.array(lo)[:, None] + rng.random((3, 200)) * (h * (np.array(dims) - 1))[:, None]
    np.testing.assert_allclose(osdf.sample(G, lo, h, dims, Q), a @ Q + 0.75, rtol=0, atol=1e-13)
    # nodes return their own values; outside the grid is +inf
    np.testing.assert_allclose(osdf.sample(G, lo, h, dims, P), G, rtol=0, atol=1e-13)
    assert np.isinf(osdf.sample(G, lo, h, dims, np.array([[-1.1], [0.5], [2.5]])))[0]
