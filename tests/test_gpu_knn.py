"""k-NN weighted surface projection on the GPU against the float64 oracle."""

import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, dev, host, scale_of
from synth import make_config
from oracle import knn as ok
from oracle import closest as oc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def _check(mg, V, F, Q, k, eps, device, max_dist2=float("inf")):
    Vd, Fd, Qd = dev(V, device), dev(F, device), dev(Q, device)
    bvh = mg.lbvh_build(Vd, Fd)
    r = mg.knn_surface_query(bvh, Vd, Qd, k=k, eps=eps, max_dist2=max_dist2)
    face, d2, pt = host(r["face"]).astype(np.int64), host(r["dist2"]).astype(np.float64), host(r["point"])
    L = scale_of(V)
    ref_f, ref_d2 = ok.knn_faces(V, F, Q, k)
    kk = ref_f.shape[0]
    ok_mask = np.isfinite(ref_d2) & (ref_d2 <= max_dist2)
    # the k smallest distances are unique: compare them
    dr, dd = np.sqrt(ref_d2), np.sqrt(d2[:kk])
    valid = face[:kk] >= 0
    np.testing.assert_array_equal(valid, ok_mask | (valid & (np.abs(dd - dr) <= 1e-5 * np.maximum(dr, 0.1 * L))))
    assert (np.abs(dd - dr)[valid] <= 1e-5 * np.maximum(dr, 0.1 * L)[valid]).all()
    # the faces may differ at ties: each device face is at its reported distance
    for j in range(kk):
        m = valid[j]
        if m.any():
            rec = oc.closest_on_faces(V, F, Q[:, m], face[j][m])
            assert (np.abs(np.sqrt(rec["dist2"]) - dd[j][m]) <= 1e-5 * np.maximum(dd[j][m], 0.1 * L)).all()
    # the weighted point from the device's faces
    full = valid.all(axis=0)
    want = ok.weighted_point(V, F, Q[:, full], face[:kk][:, full], eps)
    assert (np.abs(pt[:, full] - want) <= 1e-5 * np.maximum(np.abs(want), 0.1 * L)).all()
    return face, d2, pt


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_knn_parity_small(device, k):
    import paper_2606_00444_amd as mg
    sc = make_config(1, small=True)
    V, F = sc.frames([5])[0], sc.faces
    rng = np.random.default_rng(20 + k)
    Q = np.concatenate([sc.queries, V[:, ::9] + rng.normal(0, 1e-3, (3, V[:, ::9].shape[1])).astype(np.float32)], axis=1)
    _check(mg, V, F, Q.astype(np.float32), k, 1e-6, device)


def test_knn_k1_equals_closest_point(device):
    import paper_2606_00444_amd as mg
    sc = make_config(2, small=True)
    V, F = dev(sc.frames([3])[0], device), dev(sc.faces, device)
    Q = dev(sc.queries, device)
    bvh = mg.lbvh_build(V, F)
    a = mg.knn_surface_query(bvh, V, Q, k=1)
    b = mg.closest_point_query(bvh, V, Q)
    torch.testing.assert_close(a["face"][0], b["face"], rtol=0, atol=0)
    torch.testing.assert_close(a["dist2"][0], b["dist2"], rtol=0, atol=0)
    torch.testing.assert_close(a["point"], b["point"], rtol=0, atol=0)


def test_knn_exact_hits_and_max_dist(device):
    import paper_2606_00444_amd as mg
    sc = make_config(1, small=True)
    V, F = sc.verts0, sc.faces
    # mesh vertices are exact hits (distance 0): the point is the vertex itself, eps = 0
    Vd, Fd = dev(V, device), dev(F, device)
    bvh = mg.lbvh_build(Vd, Fd)
    r = mg.knn_surface_query(bvh, Vd, dev(V[:, ::5].copy(), device), k=4, eps=0.0)
    np.testing.assert_array_equal(host(r["point"]), V[:, ::5])
    # a radius that leaves some queries with fewer than k faces
    _check(mg, V, F, sc.queries, 4, 1e-6, device, max_dist2=0.01)


def test_knn_full_size_sampled(device):
    """The 40,000-face template (frame 7), 800 queries, k = 4."""
    import paper_2606_00444_amd as mg
    sc = make_config(2)
    rng = np.random.default_rng(8)
    Q = sc.queries[:, rng.choice(sc.queries.shape[1], 800, replace=False)]
    _check(mg, sc.frames([7])[0], sc.faces, Q, 4, 1e-6, device)
