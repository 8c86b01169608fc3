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
