"""Pins of the k-NN weighted surface projection oracle (Sec. 3.3, Eq. 1 NearestSurface)."""

import numpy as np

from oracle import knn as ok
from oracle import closest as oc
from synth.meshes import icosphere

# unit square at z = 0 split along its diagonal: T0 = (0,0)(1,0)(1,1), T1 = (0,0)(1,1)(0,1)
SQ_V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=np.float64).T
SQ_F = np.array([[0, 1, 2], [0, 2, 3]]).T


def test_k1_is_the_closest_point():
    v, f = icosphere(2)
    V, F = v.T.astype(np.float64), f.T
    rng = np.random.default_rng(0)
    Q = rng.uniform(-1.3, 1.3, (3, 300))
    r = ok.knn_surface(V, F, Q, k=1)
    c = oc.closest_point_mesh(V, F, Q)                     # the plain-C brute force
    np.testing.assert_array_equal(r["face"][0], c["face"])
    np.testing.assert_allclose(r["point"], c["point"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["dist2"][0], c["dist2"], rtol=1e-12, atol=1e-15)


def test_two_triangle_worked_example():
    # q = (0.75, 0.25, 0.5): over T0's interior, so c0 = (0.75, 0.25, 0), d0 = 0.5;
    # T1 (x <= y) is nearest on the diagonal at c1 = (0.5, 0.5, 0), d1 = sqrt(0.375).
    q = np.array([[0.75], [0.25], [0.5]])
    r = ok.knn_surface(SQ_V, SQ_F, q, k=2, eps=0.0)
    np.testing.assert_array_equal(r["face"][:, 0], [0, 1])
    np.testing.assert_allclose(r["dist2"][:, 0], [0.25, 0.375], rtol=1e-14)
    w0, w1 = 1 / 0.5, 1 / np.sqrt(0.375)
    want = (w0 * np.array([0.75, 0.25, 0]) + w1 * np.array([0.5, 0.5, 0])) / (w0 + w1)
    np.testing.assert_allclose(r["point"][:, 0], want, rtol=0, atol=1e-14)
    # more neighbours than faces: all faces, in order
    r = ok.knn_surface(SQ_V, SQ_F, q, k=5)
    np.testing.assert_array_equal(r["face"][:, 0], [0, 1])


def test_ties_go_to_the_lower_face_id_and_edge_points_agree():
    # above the diagonal's midpoint both faces are at the same distance with the same
    # closest point: any weights give that point
    q = np.array([[0.5], [0.5], [0.3]])
    r = ok.knn_surface(SQ_V, SQ_F, q, k=2, eps=1e-3)
    np.testing.assert_array_equal(r["face"][:, 0], [0, 1])
    np.testing.assert_allclose(r["point"][:, 0], [0.5, 0.5, 0.0], rtol=0, atol=1e-15)
    r1 = ok.knn_surface(SQ_V, SQ_F, q, k=1)
    np.testing.assert_array_equal(r1["face"][:, 0], [0])


def test_point_on_the_surface_is_kept():
    v, f = icosphere(2)
    V, F = v.T.astype(np.float64), f.T
    P = V[:, ::7]                                          # mesh vertices: distance 0
    r = ok.knn_surface(V, F, P, k=4, eps=0.0)
    np.testing.assert_array_equal(r["point"], P)           # the exact-hit rule
    r = ok.knn_surface(V, F, P + 1e-9, k=4, eps=1e-12)     # just off the surface
    np.testing.assert_allclose(r["point"], P, rtol=0, atol=1e-6)


def test_face_order_permutation_invariance():
    v, f = icosphere(1)
    V, F = v.T.astype(np.float64), f.T
    rng = np.random.default_rng(1)
    Q = rng.uniform(-1.2, 1.2, (3, 50))
    perm = rng.permutation(F.shape[1])
    a = ok.knn_surface(V, F, Q, k=3, eps=1e-6)
    b = ok.knn_surface(V, F[:, perm], Q, k=3, eps=1e-6)
    np.testing.assert_allclose(a["dist2"], b["dist2"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(a["point"], b["point"], rtol=0, atol=1e-12)
