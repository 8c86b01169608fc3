"""Property-based pins of the oracle (hypothesis): random inputs checked against facts
that hold for any input, so that a dropped term, a wrong sign or a swapped index in
the oracle fails somewhere.  Each property is independent of the oracle's own
formulas (optimality by sampling, invariance under rigid motions, symmetry,
exact integer identities)."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck
from hypothesis.extra.numpy import arrays

from oracle import closest as oc
from oracle import gaussians as og
from oracle import knn as ok
from oracle import lbvh as ol
from oracle import losses as olo
from oracle import morton as om

SETTINGS = dict(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
coord = st.floats(-10.0, 10.0, allow_nan=False, allow_infinity=False, width=64)
vec3 = arrays(np.float64, (3,), elements=coord)


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    return og.quat_to_matrix(q[None])[0]


def _area2(a, b, c):
    return np.linalg.norm(np.cross(b - a, c - a))


@settings(**SETTINGS)
@given(vec3, vec3, vec3, vec3)
def test_closest_point_on_triangle_is_optimal(p, a, b, c):
    """The returned point lies on the triangle (weights in [0, 1], summing to 1, reproducing
    it) and no point of a dense barycentric sample of the triangle is nearer."""
    x, w = oc.closest_on_triangle(p, a, b, c)
    assert np.all(w >= -1e-12) and np.all(w <= 1 + 1e-12)
    assert abs(w.sum() - 1) <= 1e-12
    np.testing.assert_allclose(w[0] * a + w[1] * b + w[2] * c, x, atol=1e-9 * (1 + np.abs(x).max()))
    u = np.linspace(0, 1, 41)
    U, Vv = np.meshgrid(u, u, indexing="ij")
    keep = U + Vv <= 1
    S = (1 - U[keep] - Vv[keep])[:, None] * a + U[keep][:, None] * b + Vv[keep][:, None] * c
    d_best = np.linalg.norm(p - x)
    assert d_best <= np.linalg.norm(S - p, axis=1).min() + 1e-9 * (1 + np.abs(S).max())


@settings(**SETTINGS)
@given(vec3, vec3, vec3, vec3, vec3, st.integers(0, 2**31 - 1))
def test_closest_point_is_rigid_motion_equivariant(p, a, b, c, t, seed):
    """Moving the triangle and the query by x -> R x + t moves the closest point the same way."""
    if _area2(a, b, c) < 1e-3:
        return
    R = _rotation(seed)
    x, _ = oc.closest_on_triangle(p, a, b, c)
    y, _ = oc.closest_on_triangle(R @ p + t, R @ a + t, R @ b + t, R @ c + t)
    np.testing.assert_allclose(y, R @ x + t, atol=1e-9 * (1 + np.abs(y).max()) * 1e3)


@settings(**SETTINGS)
@given(arrays(np.uint32, st.integers(2, 300), elements=st.integers(0, 2**12 - 1)))
def test_karras_tree_partitions_leaf_ranges(codes):
    """For any sorted code array (duplicates included): every internal node covers a
    contiguous leaf range split by its children, the root covers all leaves, and every
    leaf has exactly one parent."""
    codes = np.sort(codes)
    n = codes.size
    t = ol.karras_tree(codes)
    lo, hi, ch = t["lo"].astype(np.int64), t["hi"].astype(np.int64), t["child"].astype(np.int64)
    assert lo[0] == 0 and hi[0] == n - 1
    seen = np.zeros(n, int)
    for i in range(n - 1):
        rng = []
        for c in ch[:, i]:
            if c >= 0:
                rng.append((lo[c], hi[c]))
            else:
                seen[~c] += 1
                rng.append((~c, ~c))
        (l0, h0), (l1, h1) = rng
        assert l0 == lo[i] and h1 == hi[i] and h0 + 1 == l1
    assert (seen == 1).all()


@settings(**SETTINGS)
@given(arrays(np.uint32, (3, 16), elements=st.integers(0, 1023)))
def test_morton_code_is_the_digit_interleave_of_x_y_z(q):
    """The code of cell (x, y, z) read as binary digits is x9 y9 z9 x8 y8 z8 ... x0 y0 z0
    (built here from the digit strings, not from shifts), so codes increase along each axis."""
    code = (om.spread10(q[0]) << np.uint32(2)) | (om.spread10(q[1]) << np.uint32(1)) | om.spread10(q[2])
    for i in range(q.shape[1]):
        x, y, z = (format(int(v), "010b") for v in q[:, i])
        assert int(code[i]) == int("".join(a + b + c for a, b, c in zip(x, y, z)), 2)
        for axis in range(3):
            if q[axis, i] < 1023:
                r = q[:, i:i + 1].copy()
                r[axis] += 1
                up = (om.spread10(r[0]) << np.uint32(2)) | (om.spread10(r[1]) << np.uint32(1)) | om.spread10(r[2])
                assert int(up[0]) > int(code[i])


@settings(**SETTINGS)
@given(st.integers(1, 40), st.integers(1, 40), st.integers(0, 2**31 - 1))
def test_chamfer_is_symmetric_nonnegative_and_zero_on_itself(na, nb, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, na))
    B = rng.normal(size=(3, nb))
    cab = olo.chamfer(A, B)[0]
    cba = olo.chamfer(B, A)[0]
    assert cab >= 0
    assert cab == pytest.approx(cba, rel=1e-12)
    assert olo.chamfer(A, A)[0] == 0


@settings(**SETTINGS)
@given(st.integers(0, 2**31 - 1))
def test_repose_is_rigid_motion_equivariant(seed):
    """Moving every vertex by x -> R x + t moves each Gaussian's mean the same way, rotates
    its frame and turns its covariance into R S R^T; the covariance's eigenvalues stay
    exp(2 log_scale)."""
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(3, 12))
    F = np.array([[0, 3, 6, 9], [1, 4, 7, 10], [2, 5, 8, 11]])
    G = 9
    bary = rng.dirichlet([1, 1, 1], G)[:, 1:].T
    q = rng.normal(size=(4, G))
    b = {"face": rng.integers(0, 4, G), "bary": bary, "q_local": q / np.linalg.norm(q, axis=0),
         "log_scale": rng.normal(-2, 0.5, (3, G))}
    R = _rotation(seed + 1)
    t = rng.normal(size=3)
    r0 = og.repose(V, F, b)
    r1 = og.repose(R @ V + t[:, None], F, b)
    np.testing.assert_allclose(r1["mean"], R @ r0["mean"] + t[:, None], atol=1e-10)
    S0, S1 = og.unpack_sym(r0["cov"]), og.unpack_sym(r1["cov"])
    np.testing.assert_allclose(S1, np.einsum("ij,gjk,lk->gil", R, S0, R), atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(S0), axis=1)
    np.testing.assert_allclose(ev, np.sort(np.exp(2 * b["log_scale"]).T, axis=1), rtol=1e-9)


@settings(**SETTINGS)
@given(st.integers(1, 8), st.integers(0, 2**31 - 1))
def test_knn_faces_are_the_k_smallest_distances(k, seed):
    """The k faces returned are the k smallest point-to-triangle distances, sorted."""
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(3, 30))
    F = rng.integers(0, 30, (3, 20))
    Q = rng.normal(size=(3, 5))
    face, d2 = ok.knn_faces(V, F, Q, k)
    all_d = np.stack([oc.distances_to_faces(V, F, Q, np.full(5, f)) for f in range(20)])   # [F][Q]
    for qi in range(5):
        ref = np.sort(all_d[:, qi])[:k]
        np.testing.assert_allclose(d2[:, qi], ref, rtol=1e-12, atol=1e-15)
        assert np.all(np.diff(d2[:, qi]) >= 0)
