"""Seeded random meshes against the oracle: triangle soups with repeated and collinear
vertices, duplicate faces and slivers, at several scales and offsets, with queries on
vertices, on edge midpoints, near and far.  Every traversal kernel, the refit of a
perturbed frame, the slab bounds and the k-NN query are compared with the oracle."""

import numpy as np
import pytest

from gpu_helpers import need_gpu, dev, host, decode_bvh, check_slabs, scale_of
from test_gpu_query import qa
from oracle import closest as oc
from oracle import knn as ok

pytestmark = pytest.mark.gpu

KERNELS = [("lane", 0), ("batch", 1), ("seeded", 8), ("dynamic", 16)]
CASES = list(range(24))


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def soup(seed):
    """A random triangle soup (float32 vertices [3][V], int32 faces [3][F]) and queries [3][Q]."""
    rng = np.random.default_rng(7000 + seed)
    scale = [1e-2, 1.0, 1e2][seed % 3]
    offset = (5.0 * scale) if seed % 2 else 0.0
    nv = int(rng.integers(3, 160))
    V = rng.normal(0, 1, (3, nv))
    if seed % 4 == 1:                       # a flattened cloud: many near-coplanar faces
        V[2] *= 1e-3
    nf = int(rng.integers(1, 300))
    F = rng.integers(0, nv, (3, nf))
    k = nf // 5                             # repeated vertices in every position
    F[1, :k // 3] = F[0, :k // 3]
    F[2, k // 3:2 * k // 3] = F[1, k // 3:2 * k // 3]
    F[0, 2 * k // 3:k] = F[2, 2 * k // 3:k]
    if nf > 4:                              # duplicate faces, one reversed
        F[:, -1] = F[:, 0]
        F[:, -2] = F[::-1, 1]
    if nv > 6 and seed % 3 == 2:            # a collinear triple used by a face
        V[:, 3] = V[:, 1] + 0.5 * (V[:, 2] - V[:, 1])
        F[:, min(3, nf - 1)] = [1, 2, 3]
    V = (V * scale + offset).astype(np.float32)
    Vd = V.astype(np.float64)
    edge = 0.5 * (Vd[:, F[0]] + Vd[:, F[1]])
    Q = np.concatenate([
        Vd[:, rng.integers(0, nv, 40)],                                    # on vertices
        edge[:, rng.integers(0, nf, 40)],                                  # on edge midpoints
        Vd.mean(1, keepdims=True) + rng.normal(0, scale, (3, 200)),         # around the soup
        Vd.mean(1, keepdims=True) + rng.normal(0, 20 * scale, (3, 20)),     # far away
    ], axis=1).astype(np.float32)
    return V, F.astype(np.int32), Q, rng


def sin_min(V, F, fid):
    """Sine of each face's smallest angle (0 for a repeated vertex), in float64."""
    V = np.asarray(V, dtype=np.float64)
    a, b, c = (V[:, np.asarray(F)[k, fid]] for k in range(3))
    area2 = np.linalg.norm(np.cross((b - a).T, (c - a).T).T, axis=0)
    ls = [np.linalg.norm(x, axis=0) for x in (b - a, c - b, a - c)]
    prods = np.stack([ls[0] * ls[2], ls[0] * ls[1], ls[1] * ls[2]])
    return np.where(prods.max(0) > 0, area2 / np.maximum(prods.max(0), 1e-300), 0.0)


EPS32 = 2.0 ** -24


def repeated(F, fid):
    f = np.asarray(F)[:, fid]
    return (f[0] == f[1]) | (f[1] == f[2]) | (f[0] == f[2])


def soup_tol(V, F, Q, fids, d_ref):
    """Per-query tolerance: the rule for positions (1e-5 max(d, 0.1 L)) plus the float32
    evaluation bound of a closest point on a thin triangle, 8 eps32 M / sin^2 of its
    smallest angle (M the largest coordinate magnitude involved).  A face with a repeated
    vertex takes the exact segment path on both sides and keeps the plain rule."""
    L = scale_of(V)
    tol = 1e-5 * np.maximum(d_ref, 0.1 * L)
    Vd = np.abs(np.asarray(V, dtype=np.float64))
    M = np.abs(np.asarray(Q, dtype=np.float64)).max(0)
    for fid in fids:
        sm = sin_min(V, F, fid)
        thin = ~repeated(F, fid)
        Mf = np.maximum(M, Vd[:, np.asarray(F)[:, fid]].max(axis=(0, 1)))
        tol = tol + np.where(thin, 8 * EPS32 * Mf / np.maximum(sm, 1e-6) ** 2, 0.0)
    return tol


def check_soup(res, V, F, Q):
    """Closest point against the oracle with the thin-triangle bound (soup_tol): the device's
    face ties the oracle's minimum, and its distance, point and normal match the oracle's
    evaluation on that face."""
    ref = oc.closest_point_mesh(V, F, Q)
    face = host(res["face"]).astype(np.int64)
    assert (face >= 0).all()
    at = oc.closest_on_faces(V, F, Q, face)
    d_ref = np.sqrt(ref["dist2"])
    tol = soup_tol(V, F, Q, (face, ref["face"]), d_ref)
    assert (np.sqrt(at["dist2"]) <= d_ref + tol).all(), "closest face not within tie tolerance"
    d_dev = np.sqrt(host(res["dist2"]).astype(np.float64))
    assert (np.abs(d_dev - np.sqrt(at["dist2"])) <= tol).all(), "distance"
    assert (np.abs(host(res["point"]).astype(np.float64) - at["point"]).max(0) <= tol).all(), "point"
    n_dev = host(res["normal"]).astype(np.float64)
    sm = sin_min(V, F, face)
    rep = repeated(F, face)
    tol_n = 1e-5 + 1e-6 / np.maximum(sm, 1e-30)
    assert (np.abs(n_dev - at["normal"]).max(0)[~rep] <= tol_n[~rep]).all(), "normal"
    assert (n_dev[:, rep] == 0).all() and (at["normal"][:, rep] == 0).all()


def check_soup_knn(mg, V, F, Q, k, device):
    """k-NN distances against the oracle's k smallest, with the thin-triangle bound."""
    Vd = dev(V, device)
    bvh = mg.lbvh_build(Vd, dev(F, device))
    r = mg.knn_surface_query(bvh, Vd, dev(Q, device), k=k)
    face = host(r["face"]).astype(np.int64)
    d_dev = np.sqrt(host(r["dist2"]).astype(np.float64))
    ref_f, ref_d2 = ok.knn_faces(V, F, Q, k)
    for j in range(ref_f.shape[0]):
        assert (face[j] >= 0).all()
        d_ref = np.sqrt(ref_d2[j])
        tol = soup_tol(V, F, Q, (face[j], ref_f[j]), d_ref)
        assert (np.abs(d_dev[j] - d_ref) <= tol).all(), f"rank {j} distance"
        at = oc.closest_on_faces(V, F, Q, face[j])
        assert (np.abs(np.sqrt(at["dist2"]) - d_dev[j]) <= tol).all(), f"rank {j} face"


@pytest.mark.parametrize("seed", CASES)
def test_closest_point_random_soups(device, seed):
    import paper_2606_00444_amd as mg
    V, F, Q, rng = soup(seed)
    bvh = mg.lbvh_build(dev(V, device), dev(F, device))
    moved = (V + rng.normal(0, 0.05, V.shape) * np.abs(V).max()).astype(np.float32)
    for Vt in (V, moved):
        Vd = dev(Vt, device)
        mg.lbvh_refit(bvh, Vd)
        got = decode_bvh(bvh)
        assert got["status"] == 0
        check_slabs(got, Vt)
        for kernel, batch in KERNELS:
            res = mg.closest_point_query(bvh, Vd, dev(Q, device), normal=True, **qa(kernel, batch))
            check_soup(res, Vt, F, Q)


@pytest.mark.parametrize("seed", CASES[::3])
def test_knn_random_soups(device, seed):
    import paper_2606_00444_amd as mg
    V, F, Q, _ = soup(seed)
    check_soup_knn(mg, V, F, Q, 3, device)
