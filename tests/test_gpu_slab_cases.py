"""Closest-point queries on meshes that stress the normal slabs of the BVH: a flat grid
(every normal equal, slabs as thin as the rounding margin) with queries exactly on it,
faces of zero area (no normal, no slab), and two coincident sheets of opposite winding
(normal sums that cancel).  Every result is compared with the oracle, after the build
and after a refit, and every slab is checked to contain the faces below it."""

import numpy as np
import pytest

from gpu_helpers import need_gpu, dev, host, decode_bvh, check_slabs
from test_gpu_query import check_closest, qa

pytestmark = pytest.mark.gpu

KERNELS = [("lane", 0), ("batch", 8), ("seeded", 16), ("dynamic", 4)]


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def grid(nx, ny, z=0.0, flip=False):
    """A flat nx x ny grid of unit-spaced vertices in the plane z, two triangles per cell."""
    xs, ys = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), indexing="ij")
    V = np.stack([xs.ravel(), ys.ravel(), np.full(nx * ny, z)]).astype(np.float32)
    idx = np.arange(nx * ny).reshape(nx, ny)
    a, b, c, d = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    F = np.concatenate([np.stack([a, b, c]), np.stack([a, c, d])], axis=1)
    if flip:
        F = F[[0, 2, 1]]
    return V, F.astype(np.int32)


def _run(mg, device, V, F, Q, kernel, batch, frames=()):
    bvh = mg.lbvh_build(dev(V, device), dev(F, device))
    for Vt in (V,) + tuple(frames):
        Vd = dev(Vt, device)
        mg.lbvh_refit(bvh, Vd)
        got = decode_bvh(bvh)
        assert got["status"] == 0
        check_slabs(got, Vt)
        res = mg.closest_point_query(bvh, Vd, dev(Q, device), normal=True, **qa(kernel, batch))
        check_closest(res, Vt, F, Q)
        yield Vt, res


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_flat_grid_queries_on_and_off_the_plane(device, kernel, batch):
    import paper_2606_00444_amd as mg
    V, F = grid(60, 45)
    rng = np.random.default_rng(301)
    on = np.stack([rng.uniform(0, 59, 1500), rng.uniform(0, 44, 1500), np.zeros(1500)])
    off = np.stack([rng.uniform(-5, 64, 1500), rng.uniform(-5, 49, 1500), rng.normal(0, 2, 1500)])
    Q = np.concatenate([on, off, V[:, ::7].astype(np.float64)], axis=1).astype(np.float32)
    lifted = V.copy()
    lifted[2] += np.float32(0.3)
    tilted = V.copy()
    tilted[2] = (0.01 * V[0] - 0.02 * V[1]).astype(np.float32)
    for Vt, res in _run(mg, device, V, F, Q, kernel, batch, frames=(lifted, tilted)):
        if Vt is V:
            # queries inside the grid and on its plane lie on it (up to the rounding of
            # the point rebuilt from barycentrics, coordinates up to 59)
            assert np.sqrt(host(res["dist2"])[:1500].astype(np.float64)).max() <= 2e-5


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_zero_area_faces_among_regular_ones(device, kernel, batch):
    import paper_2606_00444_amd as mg
    V, F = grid(30, 30)
    rng = np.random.default_rng(302)
    V[2] = rng.normal(0, 0.2, V.shape[1]).astype(np.float32)            # a bumpy sheet
    n = V.shape[1]
    # zero-area faces: a repeated vertex, and three collinear vertices (x = row, y = 0, 1, 2, z = 0)
    deg = np.stack([np.arange(0, n - 2, 5), np.arange(0, n - 2, 5), np.arange(1, n - 1, 5)])
    row = np.arange(0, 28)
    col = np.stack([row * 30, row * 30 + 1, row * 30 + 2])
    V[2, col.ravel()] = 0.0
    Fd = np.concatenate([F, deg, col], axis=1).astype(np.int32)
    Fd = Fd[:, rng.permutation(Fd.shape[1])]
    Q = np.stack([rng.uniform(-2, 31, 3000), rng.uniform(-2, 31, 3000), rng.normal(0, 1, 3000)]).astype(np.float32)
    moved = (V + rng.normal(0, 0.05, V.shape)).astype(np.float32)
    for _ in _run(mg, device, V, Fd, Q, kernel, batch, frames=(moved,)):
        pass


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_coincident_sheets_of_opposite_winding(device, kernel, batch):
    import paper_2606_00444_amd as mg
    V, F = grid(40, 40)
    _, Ff = grid(40, 40, flip=True)
    F2 = np.concatenate([F, Ff], axis=1).astype(np.int32)                 # every cell twice, normals cancel
    rng = np.random.default_rng(303)
    Q = np.stack([rng.uniform(-3, 42, 3000), rng.uniform(-3, 42, 3000), rng.normal(0, 1.5, 3000)]).astype(np.float32)
    bent = V.copy()
    bent[2] = (0.05 * (V[0] - 20) ** 2 / 20).astype(np.float32)
    for _ in _run(mg, device, V, F2, Q, kernel, batch, frames=(bent,)):
        pass


def needles(seed):
    """A bumpy grid plus isolated faces with a repeated vertex (segments, in every vertex
    placement) and with three equal vertices (points), hanging above the grid, so that
    they are the unique nearest face of the queries around them."""
    V, F = grid(20, 20)
    rng = np.random.default_rng(seed)
    V[2] = rng.normal(0, 0.1, V.shape[1]).astype(np.float32)
    m = 60
    u = np.stack([rng.uniform(1, 18, m), rng.uniform(1, 18, m), rng.uniform(2, 4, m)])
    v = u + rng.normal(0, 0.6, (3, m))
    n0 = V.shape[1]
    V = np.concatenate([V, u.astype(np.float32), v.astype(np.float32)], axis=1)
    iu, iv = n0 + np.arange(m), n0 + m + np.arange(m)
    order = [(iu, iu, iv), (iu, iv, iu), (iv, iu, iu), (iu, iv, iv), (iv, iv, iu), (iv, iu, iv)]
    Fn = np.concatenate([np.stack(order[j % 6])[:, j:j + 1] for j in range(m)], axis=1)
    Fp = np.stack([iv[::4], iv[::4], iv[::4]])                            # point faces
    Fa = np.concatenate([F, Fn, Fp], axis=1)
    Fa = Fa[:, rng.permutation(Fa.shape[1])].astype(np.int32)
    t = rng.uniform(-0.2, 1.2, (1, 3 * m))
    Q = np.repeat(u, 3, axis=1) + t * np.repeat(v - u, 3, axis=1) + rng.normal(0, 0.15, (3, 3 * m))
    Q = np.concatenate([Q, np.stack([rng.uniform(0, 19, 500), rng.uniform(0, 19, 500),
                                     rng.uniform(-1, 5, 500)])], axis=1).astype(np.float32)
    return V, Fa, Q


@pytest.mark.parametrize("kernel,batch", KERNELS)
def test_repeated_vertex_faces_are_segments(device, kernel, batch):
    """The closest point on a face with a repeated vertex lies on the segment between its
    distinct vertices, whichever two vertices repeat, after the build and after a refit."""
    import paper_2606_00444_amd as mg
    V, F, Q = needles(304)
    moved = V.copy()
    moved[2] += np.float32(0.25)
    near = 0
    for Vt, res in _run(mg, device, V, F, Q, kernel, batch, frames=(moved,)):
        tri = F[:, host(res["face"]).astype(np.int64)]
        near += int(((tri[0] == tri[1]) | (tri[1] == tri[2]) | (tri[0] == tri[2])).sum())
    assert near >= 100                                                   # the needles were the answers


def test_repeated_vertex_faces_knn_and_nearest(device):
    import paper_2606_00444_amd as mg
    from test_gpu_knn import _check
    V, F, Q = needles(305)
    face, _, _ = _check(mg, V, F, Q, 3, 0.0, device)
    tri = F[:, np.maximum(face[0], 0)]
    assert ((tri[0] == tri[1]) | (tri[1] == tri[2]) | (tri[0] == tri[2])).sum() >= 100
