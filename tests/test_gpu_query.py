"""GPU closest-point queries (collision, template projection) against the float64 brute-force oracle."""

import math

import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, dev, host, scale_of, assert_positions
from synth import make_config
from oracle import closest as oc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def check_closest(got, verts, faces, queries, max_dist2=math.inf):
    """Face equal except ties; point, bary, distance and normal within the tolerance rule.

    The device's face must tie the oracle's minimum (its oracle distance is within
    the position tolerance of the minimum).  Two faces can tie while their closest
    points lie far apart (a query equidistant from two parts of the surface), so
    point, barycentrics, distance and normal are compared with the oracle's
    closest point on the device's face.
    """
    ref = oc.closest_point_mesh(verts, faces, queries, max_dist2=max_dist2)
    L = scale_of(verts)
    face = host(got["face"]).astype(np.int64)
    hit = ref["face"] >= 0
    if math.isinf(max_dist2):
        assert (face >= 0).all()
    assert (face[hit] >= 0).all()
    at = oc.closest_on_faces(verts, faces, queries[:, hit], face[hit])
    d_ref = np.sqrt(ref["dist2"][hit])
    tol = 1e-5 * np.maximum(d_ref, 0.1 * L)
    assert (np.sqrt(at["dist2"]) <= d_ref + tol).all(), "closest face not within tie tolerance"
    assert_positions(np.sqrt(host(got["dist2"]).astype(np.float64)[hit]), np.sqrt(at["dist2"]), L, "distance")
    assert_positions(host(got["point"])[:, hit], at["point"], L, "closest point")
    if got.get("bary") is not None:
        # the barycentrics reproduce the closest point on the device's face
        w = host(got["bary"]).astype(np.float64)[:, hit]
        tri = np.asarray(faces)[:, face[hit]]
        V = np.asarray(verts, dtype=np.float64)
        p = (1 - w[0] - w[1]) * V[:, tri[0]] + w[0] * V[:, tri[1]] + w[1] * V[:, tri[2]]
        assert_positions(p, at["point"], L, "bary point")
    if got.get("normal") is not None:
        # a unit normal from float32 vertices is accurate to about eps32 / sin(theta)
        # (theta the angle between the face's edges): a nearly degenerate face's normal
        # is set by rounding, so the bound grows as the face flattens
        n_dev = host(got["normal"]).astype(np.float64)[:, hit]
        tri = np.asarray(faces)[:, face[hit]]
        V = np.asarray(verts, dtype=np.float64)
        e1, e2 = V[:, tri[1]] - V[:, tri[0]], V[:, tri[2]] - V[:, tri[0]]
        den = np.linalg.norm(e1, axis=0) * np.linalg.norm(e2, axis=0)
        sin = np.where(den > 0, np.linalg.norm(np.cross(e1.T, e2.T).T, axis=0) / np.where(den > 0, den, 1), 0)
        tol_n = 1e-5 + 1e-6 / np.maximum(sin, 1e-30)
        assert (np.abs(n_dev - at["normal"]).max(axis=0) <= tol_n).all()
        # a face with a repeated vertex has no normal on either side, exactly
        rep = (tri[0] == tri[1]) | (tri[1] == tri[2]) | (tri[0] == tri[2])
        assert (n_dev[:, rep] == 0).all() and (at["normal"][:, rep] == 0).all()
    miss = ~hit
    if miss.any():
        assert (face[miss] == -1).all()
        assert np.isinf(host(got["dist2"])[miss]).all()
        np.testing.assert_array_equal(host(got["point"])[:, miss], queries[:, miss])
    return ref


KERNELS = [("lane", 0), ("batch", 1), ("batch", 8), ("batch", 32), ("seeded", 4), ("dynamic", 8)]


def qa(kernel, batch):
    """Traversal keyword arguments: "seeded" is the batch kernel with a greedy first descent,
    "dynamic" that kernel taking its batches from a work counter."""
    if kernel == "seeded":
        return {"kernel": "batch", "batch": batch, "seed": True}
    if kernel == "dynamic":
        return {"kernel": "batch", "batch": batch, "seed": True, "dynamic": True}
    return {"kernel": kernel, "batch": batch}


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_c1_all_queries(device, kernel, batch):
    import paper_2606_00444_amd as mg
    sc = make_config(1)
    V = sc.frames([22])[0]
    bvh = mg.lbvh_build(dev(sc.verts0, device), dev(sc.faces, device))
    Vd = dev(V, device)
    mg.lbvh_refit(bvh, Vd)
    got = mg.closest_point_query(bvh, Vd, dev(sc.queries, device), normal=True, **qa(kernel, batch))
    check_closest(got, V, sc.faces, sc.queries)


@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("batch", 8), ("seeded", 4)])
def test_c2_collision_and_template_projection_sampled(device, kernel, batch):
    import paper_2606_00444_amd as mg
    sc = make_config(2)
    V = sc.frames([71])[0]
    F = dev(sc.faces, device)
    bvh = mg.lbvh_build(dev(sc.verts0, device), F)
    Vd = dev(V, device)
    mg.lbvh_refit(bvh, Vd)
    got = mg.closest_point_query(bvh, Vd, dev(sc.queries, device), normal=True, **qa(kernel, batch))
    idx = np.random.default_rng(50).choice(sc.queries.shape[1], 1500, replace=False)
    sub = {k: (v[..., idx] if v is not None else None) for k, v in got.items()}
    check_closest(sub, V, sc.faces, sc.queries[:, idx])
    # template projection (Eq. 2): every template vertex onto the rebuilt varying target
    tv, tf = sc.target(71)
    tb = mg.lbvh_build(dev(tv, device), dev(tf, device))
    proj = mg.closest_point_query(tb, dev(tv, device), dev(sc.verts0, device), **qa(kernel, batch))
    idx = np.random.default_rng(51).choice(sc.n_verts, 1500, replace=False)
    sub = {k: (v[..., idx] if v is not None else None) for k, v in proj.items()}
    check_closest(sub, tv, tf, sc.verts0[:, idx])


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_traversal_equals_bruteforce_kernel(device, kernel, batch):
    """Every traversal gives bitwise the results of the kernel that tests every face:
    both evaluate the same closest-point routine, whose rounding does not depend on
    where it is inlined, and both break exact ties by the lowest face id."""
    import paper_2606_00444_amd as mg
    sc = make_config(2, small=True)
    tv, tf = sc.target(5)
    q = dev(sc.queries, device)
    bvh = mg.lbvh_build(dev(tv, device), dev(tf, device))
    a = mg.closest_point_query(bvh, dev(tv, device), q, normal=True, **qa(kernel, batch))
    b = mg.closest_point_bruteforce(dev(tv, device), dev(tf, device), q, normal=True)
    for k in ("face", "dist2", "point", "bary", "normal"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_queries_on_vertices_and_far_away(device, kernel, batch):
    import paper_2606_00444_amd as mg
    sc = make_config(1, small=True)
    V = sc.verts0
    bvh = mg.lbvh_build(dev(V, device), dev(sc.faces, device))
    # queries exactly on vertices: distance 0 and the vertex itself
    got = mg.closest_point_query(bvh, dev(V, device), dev(V, device), **qa(kernel, batch))
    assert (host(got["dist2"]) == 0).all()
    np.testing.assert_array_equal(host(got["point"]), V)
    check_closest(got, V, sc.faces, V)
    far = (np.random.default_rng(52).normal(size=(3, 300)) * 100).astype(np.float32)
    got = mg.closest_point_query(bvh, dev(V, device), dev(far, device), **qa(kernel, batch))
    check_closest(got, V, sc.faces, far)


@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("batch", 4), ("seeded", 2)])
def test_max_dist2_and_empty(device, kernel, batch):
    import paper_2606_00444_amd as mg
    sc = make_config(1, small=True)
    V = sc.verts0
    bvh = mg.lbvh_build(dev(V, device), dev(sc.faces, device))
    q = dev(sc.queries, device)
    got = mg.closest_point_query(bvh, dev(V, device), q, max_dist2=0.01, normal=True, **qa(kernel, batch))
    check_closest(got, V, sc.faces, sc.queries, max_dist2=0.01)
    e = mg.closest_point_query(bvh, dev(V, device), torch.empty(3, 0, device=device))
    assert e["face"].numel() == 0


@pytest.mark.parametrize("nf", [1, 2, 3])
@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("batch", 16), ("seeded", 2)])
def test_tiny_meshes(device, nf, kernel, batch):
    import paper_2606_00444_amd as mg
    rng = np.random.default_rng(60 + nf)
    V = rng.normal(size=(3, 3 * nf)).astype(np.float32)
    F = np.arange(3 * nf, dtype=np.int32).reshape(nf, 3).T.copy()
    q = rng.normal(size=(3, 500)).astype(np.float32) * 2
    bvh = mg.lbvh_build(dev(V, device), dev(F, device))
    got = mg.closest_point_query(bvh, dev(V, device), dev(q, device), normal=True, **qa(kernel, batch))
    check_closest(got, V, F, q)


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_nearest_point_query(device, kernel, batch):
    import paper_2606_00444_amd as mg
    rng = np.random.default_rng(70)
    P = rng.random((3, 30000)).astype(np.float32)
    Q = rng.random((3, 5000)).astype(np.float32)
    bvh = mg.lbvh_build(dev(P, device), None)
    idx, d2 = mg.nearest_point_query(bvh, dev(P, device), dev(Q, device), **qa(kernel, batch))
    ri, rd = oc.nearest_points(Q, P)
    idx = host(idx)
    d_dev = ((P[:, idx].astype(np.float64) - Q) ** 2).sum(0)
    assert (np.sqrt(d_dev) <= np.sqrt(rd) + 1e-5 * np.maximum(np.sqrt(rd), 0.1)).all()
    assert (idx == ri).mean() > 0.999
    assert_positions(np.sqrt(host(d2)), np.sqrt(rd), 1.0, "nn distance")


def bruteforce_all(mg, V, F, q, chunk=1 << 17):
    """The all-faces kernel over every query, in launches of `chunk` queries."""
    parts = [mg.closest_point_bruteforce(V, F, q[:, s:s + chunk].contiguous(), normal=True)
             for s in range(0, q.shape[1], chunk)]
    return {k: torch.cat([p[k] for p in parts], dim=-1) for k in parts[0]}


def assert_same_results(got, ref, what):
    for k in ("face", "dist2", "point", "bary", "normal"):
        if got.get(k) is not None:
            assert torch.equal(got[k], ref[k]), (what, k)


@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("batch", 8), ("seeded", 4), ("batch", 16)])
def test_c5_large(device, kernel, batch):
    """The 500,000-face template (frame 37) with all 1,000,000 queries: every result
    bitwise equal to the all-faces kernel, and 1,000 sampled queries against the oracle.
    Batches of 16 take the five-wave register allocation at this size."""
    import paper_2606_00444_amd as mg
    sc = make_config(5)
    F = dev(sc.faces, device)
    bvh = mg.lbvh_build(dev(sc.verts0, device), F)
    V = sc.frames([37])[0]
    Vd = dev(V, device)
    mg.lbvh_refit(bvh, Vd)
    q = dev(sc.queries, device)
    got = mg.closest_point_query(bvh, Vd, q, normal=True, **qa(kernel, batch))
    assert_same_results(got, bruteforce_all(mg, Vd, F, q), "C5 template")
    idx = np.random.default_rng(80).choice(sc.queries.shape[1], 1000, replace=False)
    sub = {k: (v[..., idx] if v is not None else None) for k, v in got.items()}
    check_closest(sub, V, sc.faces, sc.queries[:, idx])


def test_c5_rebuilt_target(device):
    """The 1,000,000-face varying-topology target of frame 21, rebuilt: all 1,000,000
    queries bitwise equal to the all-faces kernel, 1,000 sampled against the oracle."""
    import paper_2606_00444_amd as mg
    sc = make_config(5)
    tv, tf = sc.target(21)
    Tv, Tf = dev(tv, device), dev(tf, device)
    bvh = mg.lbvh_build(Tv, Tf)
    q = dev(sc.queries, device)
    got = mg.closest_point_query(bvh, Tv, q, normal=True, kernel="batch", batch=16, seed=True)
    assert_same_results(got, bruteforce_all(mg, Tv, Tf, q), "C5 target")
    idx = np.random.default_rng(81).choice(sc.queries.shape[1], 1000, replace=False)
    sub = {k: (v[..., idx] if v is not None else None) for k, v in got.items()}
    check_closest(sub, tv, tf, sc.queries[:, idx])


def test_c2_bench_options_full_size(device):
    """The traversal options the C2 benchmark runs with (batches of 16 with the seed
    descent; collision queries started from the previous frame's faces; template
    projection in batches of 8) at full size: every query bitwise equal to the
    all-faces kernel, 2,000 sampled queries of each set against the oracle."""
    import paper_2606_00444_amd as mg
    sc = make_config(2)
    F = dev(sc.faces, device)
    bvh = mg.lbvh_build(dev(sc.verts0, device), F)
    q = dev(sc.queries, device)
    rng = np.random.default_rng(82)
    V0 = dev(sc.frames([120])[0], device)
    mg.lbvh_refit(bvh, V0)
    prev = mg.closest_point_query(bvh, V0, q, kernel="batch", batch=16, seed=True)["face"].clone()
    V = sc.frames([121])[0]
    Vd = dev(V, device)
    mg.lbvh_refit(bvh, Vd)
    got = mg.closest_point_query(bvh, Vd, q, normal=True, kernel="batch", batch=16, seed=True, hint=prev)
    assert_same_results(got, bruteforce_all(mg, Vd, F, q), "collision")
    idx = rng.choice(sc.queries.shape[1], 2000, replace=False)
    check_closest({k: (v[..., idx] if v is not None else None) for k, v in got.items()}, V, sc.faces,
                  sc.queries[:, idx])
    tv, tf = sc.target(121)
    Tv, Tf = dev(tv, device), dev(tf, device)
    tb = mg.lbvh_build(Tv, Tf)
    for name, qq, qn, opts in (("collision vs target", q, sc.queries, {"batch": 16}),
                               ("projection", dev(sc.verts0, device), sc.verts0, {"batch": 8})):
        got = mg.closest_point_query(tb, Tv, qq, normal=True, kernel="batch", seed=True, **opts)
        assert_same_results(got, bruteforce_all(mg, Tv, Tf, qq), name)
        idx = rng.choice(qn.shape[1], 2000, replace=False)
        check_closest({k: (v[..., idx] if v is not None else None) for k, v in got.items()}, tv, tf, qn[:, idx])


@pytest.mark.parametrize("batch", [2, 8, 16])
def test_register_allocations_agree(device, batch):
    """The batch kernel's four- and five-wave register allocations (forced, and chosen
    by launch size) give bitwise the same results, which match the oracle."""
    import paper_2606_00444_amd as mg
    import torch
    sc = make_config(2, small=True)
    V = sc.frames([11])[0]
    Vd, F, q = dev(V, device), dev(sc.faces, device), dev(sc.queries, device)
    bvh = mg.lbvh_build(Vd, F)
    runs = {w: mg.closest_point_query(bvh, Vd, q, normal=True, kernel="batch", batch=batch, seed=True, waves=w)
            for w in (0, 4, 5)}
    for w in (4, 5):
        for k in ("face", "dist2", "point", "bary", "normal"):
            assert torch.equal(runs[w][k], runs[0][k]), (w, k)
    check_closest(runs[5], V, sc.faces, sc.queries)


@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("batch", 8), ("seeded", 4)])
def test_query_order_and_counters(device, kernel, batch):
    import paper_2606_00444_amd as mg
    sc = make_config(2, small=True)
    V = sc.frames([9])[0]
    Vd, F, q = dev(V, device), dev(sc.faces, device), dev(sc.queries, device)
    bvh = mg.lbvh_build(Vd, F)
    order = mg.query_order(q)
    # a permutation of the query indices
    np.testing.assert_array_equal(np.sort(host(order)), np.arange(q.shape[1]))
    cnt = torch.zeros(4, dtype=torch.int64, device=device)
    a = mg.closest_point_query(bvh, Vd, q, **qa(kernel, batch))
    b = mg.closest_point_query(bvh, Vd, q, order=order, counters=cnt, **qa(kernel, batch))
    # results land at each query's own index whatever the processing order, bitwise
    for k in ("face", "dist2", "point"):
        assert torch.equal(a[k], b[k]), k
    check_closest(b, V, sc.faces, sc.queries)
    c = host(cnt)
    assert c[3] == q.shape[1]
    assert c[0] >= q.shape[1] and 0 < c[2] <= c[1]


def test_autotuner_picks_a_valid_traversal(device, tmp_path, monkeypatch):
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd import autotune
    monkeypatch.setenv("MGU_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sc = make_config(1, small=True)
    Vd, q = dev(sc.verts0, device), dev(sc.queries, device)
    bvh = mg.lbvh_build(Vd, dev(sc.faces, device))
    res = autotune.tune_closest(bvh, Vd, q, reps=2)
    assert res["kernel"] in ("lane", "batch") and len(res["timings"]) == len(autotune.CANDIDATES)
    assert res["order"] == "given"
    assert autotune.tune_closest(bvh, Vd, q, reps=2) == res       # cached
    got = mg.closest_point_query(bvh, Vd, q, **autotune.options(res))
    check_closest(got, sc.verts0, sc.faces, sc.queries)


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_hints_do_not_change_results(device, kernel, batch):
    """Starting queries from hinted faces (the previous frame's answers, random ids, -1,
    out-of-range ids, and the output array itself as the hint) gives bitwise the
    results of the unhinted traversal."""
    import paper_2606_00444_amd as mg
    import torch
    sc = make_config(2, small=True)
    F = dev(sc.faces, device)
    bvh = mg.lbvh_build(dev(sc.verts0, device), F)
    Q = dev(sc.queries, device)
    nq, nf = sc.queries.shape[1], sc.faces.shape[1]
    mg.lbvh_refit(bvh, dev(sc.frames([9])[0], device))
    prev = mg.closest_point_query(bvh, dev(sc.frames([9])[0], device), Q, **qa(kernel, batch))["face"].clone()
    V = dev(sc.frames([10])[0], device)
    mg.lbvh_refit(bvh, V)
    base = mg.closest_point_query(bvh, V, Q, normal=True, **qa(kernel, batch))
    rng = np.random.default_rng(404)
    hints = {
        "previous frame": prev,
        "random": torch.from_numpy(rng.integers(0, nf, nq).astype(np.int32)).to(device),
        "none": torch.full((nq,), -1, dtype=torch.int32, device=device),
        "mixed, out of range": torch.from_numpy(rng.integers(-5, nf + 5, nq).astype(np.int32)).to(device),
    }
    for name, h in hints.items():
        got = mg.closest_point_query(bvh, V, Q, normal=True, hint=h, **qa(kernel, batch))
        for k in ("face", "dist2", "point", "bary", "normal"):
            assert torch.equal(got[k], base[k]), (name, k)
    # the output face array as its own hint (each query reads its hint before writing)
    out = {k: (v.clone() if v is not None else None) for k, v in base.items()}
    out["face"].copy_(prev)
    got = mg.closest_point_query(bvh, V, Q, normal=True, out=out, hint=out["face"], **qa(kernel, batch))
    for k in ("face", "dist2", "point", "bary", "normal"):
        assert torch.equal(got[k], base[k]), ("aliased", k)


@pytest.mark.parametrize("kernel,batch", [("lane", 0), ("seeded", 8)])
def test_nearest_point_hints(device, kernel, batch):
    import paper_2606_00444_amd as mg
    import torch
    rng = np.random.default_rng(405)
    P = rng.random((3, 20000)).astype(np.float32)
    q = rng.random((3, 5000)).astype(np.float32)
    bvh = mg.lbvh_build(dev(P, device), None)
    idx, d2 = mg.nearest_point_query(bvh, dev(P, device), dev(q, device), **qa(kernel, batch))
    h = torch.from_numpy(rng.integers(-3, 20003, 5000).astype(np.int32)).to(device)
    idx2, d22 = mg.nearest_point_query(bvh, dev(P, device), dev(q, device), hint=h, **qa(kernel, batch))
    assert torch.equal(idx, idx2) and torch.equal(d2, d22)


def test_chamfer_warm_start(device):
    """Chamfer started from earlier nearest-neighbour arrays (valid, absent and out-of-range
    ids, of their own direction's lengths) gives bitwise the cold results."""
    import paper_2606_00444_amd as mg
    import torch
    rng = np.random.default_rng(406)
    a = dev(rng.normal(size=(3, 3000)).astype(np.float32), device)
    b = dev(rng.normal(size=(3, 2000)).astype(np.float32), device)
    bvh_a, bvh_b = mg.lbvh_build(a, None), mg.lbvh_build(b, None)
    base = mg.chamfer(a, bvh_a, b, bvh_b)
    out = {"nn_ab": torch.from_numpy(rng.integers(-3, 2003, 3000).astype(np.int32)).to(device),
           "nn_ba": torch.from_numpy(rng.integers(-3, 3003, 2000).astype(np.int32)).to(device)}
    got = mg.chamfer(a, bvh_a, b, bvh_b, out=out, warm=True)
    for k in ("nn_ab", "d_ab", "nn_ba", "d_ba", "means"):
        assert torch.equal(got[k], base[k]), k
    # a second warm call from its own answers
    again = mg.chamfer(a, bvh_a, b, bvh_b, out=got, warm=True)
    for k in ("nn_ab", "d_ab", "nn_ba", "d_ba", "means"):
        assert torch.equal(again[k], base[k]), k
