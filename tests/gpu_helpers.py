"""Shared helpers for the GPU parity tests: device transfer, BVH decoding, tolerances.

The tolerance rule (float32 device vs float64 oracle), with L the diagonal-scale
of the frame's mesh (largest bounding-box extent):
  positions, means, distances  |d| <= 1e-5 * max(|ref|, 0.1 L)
  covariance entries           |d| <= 1e-5 * ||Sigma_ref||_F
  quaternions                  min(|q - q_ref|, |q + q_ref|) <= 1e-5
  boxes, codes, permutations, topology: bitwise
  face ids: bitwise except ties (the oracle distance to the device's face is
  within the position tolerance of the oracle's minimum).
"""

import numpy as np
import pytest
import torch

REL = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_00444_amd as mg
    mg.check_device()          # raises if libmgu.so is missing or the device is not gfx950
    return torch.device("cuda:0")


def dev(a, device):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def host(t):
    return t.detach().cpu().numpy()


def scale_of(verts):
    v = np.asarray(verts, dtype=np.float64)
    return float(np.ptp(v, axis=1).max())


def assert_positions(got, ref, L, what="positions"):
    got = np.asarray(got, dtype=np.float64)
    tol = REL * np.maximum(np.abs(ref), 0.1 * L)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{what}: {bad.sum()} entries off, worst {np.max(np.abs(got - ref) / tol):.3g}x tol"


def assert_quats(got, ref):
    got = np.asarray(got, dtype=np.float64)
    d = np.minimum(np.linalg.norm(got - ref, axis=0), np.linalg.norm(got + ref, axis=0))
    assert d.max() <= REL, f"quaternions off by {d.max():.3g}"


def assert_cov(got, ref):
    got = np.asarray(got, dtype=np.float64)
    # Frobenius norm of the symmetric matrix from its packed entries
    fro = np.sqrt(ref[0] ** 2 + ref[3] ** 2 + ref[5] ** 2 + 2 * (ref[1] ** 2 + ref[2] ** 2 + ref[4] ** 2))
    bad = np.abs(got - ref) > REL * fro[None]
    assert not bad.any(), f"covariance: {bad.sum()} entries off"


def decode_bvh(bvh):
    """Host copy of a device LBVH: codes, prim, topology and per-node boxes (Karras numbering)."""
    n = bvh.n
    m = max(n - 1, 0)
    out = {
        "codes": host(bvh.section("codes", torch.int32, n)).view(np.uint32),
        "prim": host(bvh.section("prim", torch.int32, n)),
        "leaf_parent": host(bvh.section("leaf_parent", torch.int32, n)),
        "node_parent": host(bvh.section("node_parent", torch.int32, m)),
    }
    if bvh.kind == 0:
        out["leaf_faces"] = host(bvh.section("leaf_faces", torch.int32, 3 * n)).reshape(3, n)
    hdr = host(bvh.buf[:256].view(torch.float32))
    hdr_i = host(bvh.buf[:256].view(torch.int32))
    out["n_prims"], out["status"] = int(hdr_i[0]), int(hdr_i[2])
    root = np.concatenate([hdr[4:7], hdr[8:11]]).astype(np.float64)
    out["root_box"] = root
    nodes = host(bvh.section("nodes", torch.float32, 24 * m)).reshape(m, 2, 3, 4)   # [node][slot][f4][xyzw]
    ints = nodes.view(np.int32)
    out["child"] = np.stack([ints[:, 0, 0, 3], ints[:, 1, 0, 3]]) if m else np.zeros((2, 0), np.int32)
    out["aux"] = np.stack([ints[:, 0, 1, 3], ints[:, 1, 1, 3]]) if m else np.zeros((2, 0), np.int32)
    # box of the child in each slot: a leaf triangle's min/max, else (lo, hi) of the first two float4
    xyz = nodes[:, :, :, :3].astype(np.float64)                                      # [m][2][3][3]
    leaf = (ints[:, :, 0, 3] < 0)[..., None]
    if bvh.kind == 0:
        lo = np.where(leaf, xyz.min(axis=2), xyz[:, :, 0])
        hi = np.where(leaf, xyz.max(axis=2), xyz[:, :, 1])
    else:
        lo, hi = xyz[:, :, 0], xyz[:, :, 1]
    slot_box = np.concatenate([lo, hi], axis=2)                                        # [m][2][6]
    if m:
        # leaf slots carry the primitive itself: triangle vertices (or the point) bitwise
        out["slot_vertices"] = xyz
    ib = np.zeros((m, 6))
    lb = np.zeros((n, 6))
    if m:
        ib[0] = root
        np_ = out["node_parent"]
        c = np.arange(1, m)
        ib[c] = slot_box[np_[c] >> 1, np_[c] & 1]
        lp = out["leaf_parent"]
        lb[:] = slot_box[lp >> 1, lp & 1]
    elif n == 1:
        lb[0] = root
    out["internal_box"], out["leaf_box"] = ib, lb
    if bvh.kind == 0 and m:
        # normal slab of the internal child in each slot: direction (float4 2 .xyz), a (float4 1 .w), b (float4 2 .w)
        out["slab_dir"] = nodes[:, :, 2, :3].astype(np.float64)
        out["slab_a"] = nodes[:, :, 1, 3].astype(np.float64)
        out["slab_b"] = nodes[:, :, 2, 3].astype(np.float64)
    return out


def check_slabs(got, verts):
    """Every vertex of every face below an internal child lies inside that child's stored
    slab, a <= d.x <= b, evaluated in float64 on the stored float32 values (no tolerance):
    walks each leaf up through all of its internal ancestors."""
    V = np.asarray(verts, dtype=np.float64)
    n = got["prim"].size
    if n < 3:
        return 0
    tri = V[:, got["leaf_faces"]]                          # [3 coord][3 vert][n]
    node_parent = got["node_parent"]
    cur = got["leaf_parent"] >> 1                           # each leaf's parent (an internal node)
    leaves = np.arange(n)
    checked = 0
    for _ in range(70):
        live = cur > 0                                      # the root (node 0) has no slab
        if not live.any():
            break
        c = cur[live]
        tag = node_parent[c]
        ps, sl = tag >> 1, tag & 1
        d = got["slab_dir"][ps, sl]                         # [k][3]
        a, b = got["slab_a"][ps, sl], got["slab_b"][ps, sl]
        x = tri[:, :, leaves[live]]                         # [3][3][k]
        proj = np.einsum("kc,cvk->vk", d, x)
        assert np.all(a[None] <= proj) and np.all(proj <= b[None]), "a vertex lies outside a slab"
        assert np.all(np.isfinite(a) | (np.linalg.norm(d, axis=1) == 0))
        checked += c.size
        nxt = node_parent[c] >> 1
        cur = cur.copy()
        cur[live] = np.where(tag < 0, 0, nxt)
    return checked


def check_knn_result(r, V, F, Q, k, eps, max_dist2=float("inf")):
    """A k-NN weighted projection result r (device dict: face [k][Q], dist2 [k][Q],
    point [3][Q]) of queries Q on mesh (V, F) against the float64 oracle, exactly
    where ties leave no choice: the k smallest distances match the oracle's (they are
    unique even when the faces are not), every device face lies at its reported
    distance, and the device point is the weighted point of the device's own faces."""
    from oracle import knn as ok
    from oracle import closest as oc
    face, d2, pt = host(r["face"]).astype(np.int64), host(r["dist2"]).astype(np.float64), host(r["point"])
    L = scale_of(V)
    ref_f, ref_d2 = ok.knn_faces(V, F, Q, k)
    kk = ref_f.shape[0]
    ok_mask = np.isfinite(ref_d2) & (ref_d2 <= max_dist2)
    dr, dd = np.sqrt(ref_d2), np.sqrt(d2[:kk])
    valid = face[:kk] >= 0
    np.testing.assert_array_equal(valid, ok_mask | (valid & (np.abs(dd - dr) <= REL * np.maximum(dr, 0.1 * L))))
    assert (np.abs(dd - dr)[valid] <= REL * np.maximum(dr, 0.1 * L)[valid]).all()
    for j in range(kk):
        m = valid[j]
        if m.any():
            rec = oc.closest_on_faces(V, F, Q[:, m], face[j][m])
            assert (np.abs(np.sqrt(rec["dist2"]) - dd[j][m]) <= REL * np.maximum(dd[j][m], 0.1 * L)).all()
    full = valid.all(axis=0)
    want = ok.weighted_point(V, F, Q[:, full], face[:kk][:, full], eps)
    # The weighted point P = sum w_i c_i / W, w_i = 1 / (d_i + eps), moves by
    # dP/dd_i = -w_i^2 (c_i - P) / W under an error in d_i; a float32 distance is off
    # by a few units in the last place of the coordinates' magnitude M, so when one
    # face is far nearer than the others that rounding is amplified.  The bound adds
    # 8 eps32 M times that sensitivity to the position rule.
    recs = [oc.closest_on_faces(V, F, Q[:, full], face[j][full]) for j in range(kk)]
    dist = np.stack([np.sqrt(r["dist2"]) for r in recs])                       # [k][Q']
    with np.errstate(divide="ignore"):
        w = np.where(dist + eps > 0, 1.0 / (dist + eps), 0.0)
    W = w.sum(axis=0)
    sens = np.zeros(dist.shape[1])
    for j, r in enumerate(recs):
        sens += w[j] ** 2 * np.linalg.norm(r["point"] - want, axis=0)
    sens = np.where(W > 0, sens / np.where(W > 0, W, 1.0), 0.0)
    M = float(np.abs(np.asarray(V, dtype=np.float64)).max())
    # each closest point c_i is itself only as accurate as its triangle allows: the
    # float32 bound 8 eps32 M / sin^2 of the smallest angle (thin marching-tetrahedra
    # triangles), weighted by the face's share w_i / W of the combination
    thin = np.zeros(dist.shape[1])
    for j in range(kk):
        thin += w[j] * 8 * 2.0 ** -24 * M / np.maximum(sin_smallest_angle(V, F, face[j][full]), 1e-30) ** 2
    thin = np.where(W > 0, thin / np.where(W > 0, W, 1.0), 0.0)
    tol = REL * np.maximum(np.abs(want), 0.1 * L) + 8 * 2.0 ** -24 * M * sens[None] + thin[None]
    assert (np.abs(pt[:, full] - want) <= tol).all()
    return face, d2, pt


def sin_smallest_angle(V, F, face_ids):
    """Sine of the smallest interior angle of each given face (0 for a degenerate one)."""
    V = np.asarray(V, dtype=np.float64)
    tri = np.asarray(F)[:, np.asarray(face_ids, dtype=np.int64)]
    P = [V[:, tri[k]] for k in range(3)]
    out = np.full(tri.shape[1], np.inf)
    for x, y, z in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        u, v = P[y] - P[x], P[z] - P[x]
        den = np.linalg.norm(u, axis=0) * np.linalg.norm(v, axis=0)
        sn = np.where(den > 0, np.linalg.norm(np.cross(u.T, v.T).T, axis=0) / np.where(den > 0, den, 1.0), 0.0)
        out = np.minimum(out, sn)
    return out
