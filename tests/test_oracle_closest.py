"""Pins of the oracle's closest-point routines (CPU only)."""

import json
import os

import numpy as np
import pytest

from oracle import closest as oc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def kkt_closest(p, a, b, c):
    """Independent closest point: minimise |p - x|^2 over the triangle by enumerating
    the KKT candidates - the unconstrained plane minimiser (2x2 normal equations)
    if it lies inside, the three clamped edge projections, the three vertices."""
    cands = []
    e1, e2 = b - a, c - a
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    if abs(np.linalg.det(G)) > 0:
        u, v = np.linalg.solve(G, np.array([(p - a) @ e1, (p - a) @ e2]))
        if u >= 0 and v >= 0 and u + v <= 1:
            cands.append(a + u * e1 + v * e2)
    for s, t in ((a, b), (a, c), (b, c)):
        d = t - s
        x = np.clip((p - s) @ d / (d @ d), 0, 1) if d @ d > 0 else 0.0
        cands.append(s + x * d)
    cands += [a, b, c]
    d2 = [((p - x) ** 2).sum() for x in cands]
    return min(d2)


def test_golden_regions():
    gold = json.load(open(os.path.join(GOLD, "ericson_regions.json")))
    a, b, c = (np.array(x, dtype=np.float64) for x in gold["triangle"])
    for case in gold["cases"]:
        p = np.array(case["p"], dtype=np.float64)
        pt, w = oc.closest_on_triangle(p, a, b, c)
        np.testing.assert_allclose(pt, case["c"], atol=1e-15, err_msg=case["region"])
        np.testing.assert_allclose(w, case["w"], atol=1e-15, err_msg=case["region"])
        assert ((p - pt) ** 2).sum() == pytest.approx(case["d2"], abs=1e-14)


def test_against_kkt_enumeration():
    rng = np.random.default_rng(20)
    for _ in range(2000):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2
        pt, w = oc.closest_on_triangle(p, a, b, c)
        d2 = ((p - pt) ** 2).sum()
        ref = kkt_closest(p, a, b, c)
        assert d2 == pytest.approx(ref, rel=1e-12, abs=1e-14)
        np.testing.assert_allclose(w.sum(), 1.0, atol=1e-12)
        assert (w >= -1e-12).all()
        np.testing.assert_allclose(w[0] * a + w[1] * b + w[2] * c, pt, atol=1e-12)


def test_dense_barycentric_grid():
    rng = np.random.default_rng(21)
    u = np.linspace(0, 1, 301)
    U, W = np.meshgrid(u, u)
    m = U + W <= 1
    U, W = U[m], W[m]
    for _ in range(20):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3)
        pts = a + U[:, None] * (b - a) + W[:, None] * (c - a)
        brute = ((pts - p) ** 2).sum(1).min()
        pt, _ = oc.closest_on_triangle(p, a, b, c)
        d2 = ((p - pt) ** 2).sum()
        assert d2 <= brute + 1e-12
        assert brute - d2 < 1e-3 * (1 + brute)


def test_vertex_query_exact_and_projection():
    rng = np.random.default_rng(22)
    a, b, c = rng.normal(size=(3, 3))
    for k, v in enumerate((a, b, c)):
        pt, w = oc.closest_on_triangle(v, a, b, c)
        np.testing.assert_array_equal(pt, v)
        assert w[k] == 1.0
    # point above the interior projects orthogonally
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n)
    inner = (a + b + c) / 3
    pt, _ = oc.closest_on_triangle(inner + 0.7 * n, a, b, c)
    np.testing.assert_allclose(pt, inner, atol=1e-12)


def test_zero_area_triangle_uses_segments():
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([3.0, 0, 0])
    for p in (np.array([2.0, 1.0, 0.0]), np.array([-1.0, 0.5, 0.2]), np.array([4.0, 0.0, 1.0])):
        pt, w = oc.closest_on_triangle(p, a, b, c)
        q = np.array([np.clip(p[0], 0, 3), 0, 0])
        np.testing.assert_allclose(pt, q, atol=1e-15)
        np.testing.assert_allclose(w[0] * a + w[1] * b + w[2] * c, pt, atol=1e-15)


def test_repeated_vertex_triangles_are_segments():
    """A triangle with two equal vertices is the segment between the distinct ones (or a
    point): the nearest point is the clamped projection onto that segment, whichever two
    vertices repeat, and both codings of the mesh query find it as the unique nearest."""
    u, v = np.array([0.0, 0, 0]), np.array([2.0, 0, 0])
    P = np.array([[1.0, 1.0, 0.0], [0.5, -0.3, 0.4], [-1.0, 0.2, 0.0], [3.0, 0.0, 1.0]])
    want = np.stack([np.clip(P[:, 0], 0, 2), np.zeros(4), np.zeros(4)], axis=1)
    for tri in ((u, u, v), (u, v, u), (v, u, u), (u, v, v), (v, v, u), (v, u, v)):
        for p, q in zip(P, want):
            pt, w = oc.closest_on_triangle(p, *tri)
            np.testing.assert_allclose(pt, q, atol=1e-15)
            np.testing.assert_allclose(w.sum(), 1.0, atol=1e-15)
    pt, _ = oc.closest_on_triangle(P[0], u, u, u)                       # all three equal: the point
    np.testing.assert_array_equal(pt, u)
    # mesh: one proper triangle far away, and the six degenerate faces
    verts = np.array([[0.0, 2.0, 50, 51, 50], [0, 0, 50, 50, 51], [0, 0, 0, 0, 0]])
    faces = np.array([[2, 0, 0, 1, 0, 1, 1], [3, 0, 1, 0, 1, 1, 0], [4, 1, 0, 0, 1, 0, 1]])
    for impl in ("c", "numpy"):
        r = oc.closest_point_mesh(verts, faces, P.T, impl=impl)
        np.testing.assert_array_equal(r["face"], [1, 1, 1, 1])            # lowest of the tied faces
        np.testing.assert_allclose(r["point"], want.T, atol=1e-15)
        np.testing.assert_allclose(r["dist2"], ((P - want) ** 2).sum(1), rtol=1e-15)


def test_mesh_closest_cube_and_ties():
    # unit cube, 12 faces; a query far along +x lands on the x = 1 side
    V = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=np.float64).T
    F = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                  [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]]).T
    q = np.array([[3.0, 0.3, 0.6], [0.5, 0.5, 0.5], [1.0, 1.0, 1.0]]).T
    r = oc.closest_point_mesh(V, F, q)
    np.testing.assert_allclose(r["point"][:, 0], [1.0, 0.3, 0.6], atol=1e-15)
    assert r["dist2"][0] == pytest.approx(4.0)
    assert F[:, r["face"][0]].tolist() in ([4, 6, 7], [4, 7, 5])
    # the cube centre is equidistant (0.25) to every face: lowest face id wins
    assert r["face"][1] == 0 and r["dist2"][1] == pytest.approx(0.25)
    # a corner vertex is on many faces: lowest id containing vertex 7 wins
    assert r["face"][2] == 2 and r["dist2"][2] == 0.0
    np.testing.assert_allclose(r["normal"][:, 0], [1, 0, 0], atol=1e-15)
    # nothing within max_dist2
    r = oc.closest_point_mesh(V, F, q, max_dist2=0.1)
    assert r["face"][0] == -1 and np.isinf(r["dist2"][0])
    np.testing.assert_array_equal(r["point"][:, 0], q[:, 0])


def test_mesh_closest_matches_per_face_minimum():
    from synth import make_config
    sc = make_config(1, small=True)
    V, F = sc.verts0, sc.faces
    q = sc.queries[:, :50]
    r = oc.closest_point_mesh(V, F, q)
    for i in range(0, 50, 5):
        d = oc.distances_to_faces(V, F, np.repeat(q[:, i:i + 1], F.shape[1], 1), np.arange(F.shape[1]))
        assert r["dist2"][i] == d.min()
        assert r["face"][i] == np.argmin(d)


def test_template_projection_identity():
    # projecting a mesh's own vertices onto itself returns them unchanged
    from synth import make_config
    sc = make_config(2, small=True)
    pts, r = oc.template_projection(sc.verts0, sc.verts0, sc.faces)
    np.testing.assert_array_equal(pts, sc.verts0.astype(np.float64))
    assert (r["dist2"] == 0).all()


def test_nearest_points_vs_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(23)
    A, B = rng.random((3, 3000)), rng.random((3, 2000))
    idx, d2 = oc.nearest_points(A, B)
    dk, ik = cKDTree(B.T).query(A.T)
    np.testing.assert_allclose(d2, dk ** 2, rtol=1e-12)
    np.testing.assert_array_equal(idx, ik)


def test_c_and_numpy_codings_agree():
    from synth import make_config
    sc = make_config(2, small=True)
    tv, tf = sc.target(33)
    q = sc.queries[:, :300]
    a = oc.closest_point_mesh(tv, tf, q, impl="c")
    b = oc.closest_point_mesh(tv, tf, q, impl="numpy")
    np.testing.assert_array_equal(a["face"], b["face"])
    np.testing.assert_allclose(a["dist2"], b["dist2"], rtol=1e-13)
    np.testing.assert_allclose(a["point"], b["point"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(a["bary"], b["bary"], rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(a["normal"], b["normal"])
    ia, da = oc.nearest_points(q, tv, impl="c")
    ib, db = oc.nearest_points(q, tv, impl="numpy")
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_allclose(da, db, rtol=1e-14)
