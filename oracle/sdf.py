"""Index signed-distance grid (the SDF of Sec. 3.4, Initialization), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper builds its acceleration structures (a BVH and an SDF) once from the
template faces, storing only vertex and face indices so that they serve every
frame.  Reading for the SDF: a regular grid whose nodes store, at
initialisation, the ids of their k nearest template faces; at every frame a
node's signed distance is recomputed from those faces' current vertices: the
minimum point-to-triangle distance over them, signed by the winning face's
normal (positive on the side the normal points to, zero distance counts as
positive), ties to the lowest slot.  Queries interpolate the grid trilinearly;
outside the grid the value is +inf.  It is exact while a node's nearest face
stays among its k stored faces, and an upper bound of the unsigned distance
otherwise.  Parity with the paper is unpinned (it gives no construction).
"""

import numpy as np

from .closest import closest_on_faces


def grid_points(lo, h, dims):
    """Node positions [3][nx*ny*nz], x fastest: node (i, j, k) at lo + h (i, j, k)."""
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([lo[0] + h * i.ravel(), lo[1] + h * j.ravel(), lo[2] + h * k.ravel()]).astype(np.float64)


def sdf_from_faces(verts, faces, points, face_k):
    """Signed distance of points [3][N] over their candidate faces face_k [k][N]:
    dict sdf [N], face [N] (the winning face)."""
    face_k = np.asarray(face_k, dtype=np.int64)
    P = np.asarray(points, dtype=np.float64)
    best = np.full(P.shape[1], np.inf)
    sgn = np.ones(P.shape[1])
    win = np.full(P.shape[1], -1, np.int64)
    for j in range(face_k.shape[0]):
        ok = face_k[j] >= 0
        if not ok.any():
            continue
        r = closest_on_faces(verts, faces, P[:, ok], face_k[j][ok])
        d2 = r["dist2"]
        better = d2 < best[ok]
        idx = np.nonzero(ok)[0][better]
        best[idx] = d2[better]
        win[idx] = face_k[j][ok][better]
        side = ((P[:, ok] - r["point"]) * r["normal"]).sum(0)
        sgn[idx] = np.where(side[better] >= 0, 1.0, -1.0)
    return {"sdf": sgn * np.sqrt(best), "face": win}


def sample(sdf, lo, h, dims, queries):
    """Trilinear interpolation of the node values sdf [nx*ny*nz] at queries [3][Q]; +inf outside."""
    nx, ny, nz = dims
    G = np.asarray(sdf, dtype=np.float64).reshape(nz, ny, nx)
    Q = np.asarray(queries, dtype=np.float64)
    u = (Q - np.asarray(lo, dtype=np.float64)[:, None]) / h
    out = np.full(Q.shape[1], np.inf)
    inside = ((u >= 0) & (u <= np.array([nx - 1, ny - 1, nz - 1])[:, None])).all(0)
    ui = u[:, inside]
    i0 = np.minimum(np.floor(ui).astype(np.int64), np.array([nx - 2, ny - 2, nz - 2])[:, None])
    t = ui - i0
    acc = np.zeros(ui.shape[1])
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((t[0] if dx else 1 - t[0]) * (t[1] if dy else 1 - t[1]) * (t[2] if dz else 1 - t[2]))
                acc += w * G[i0[2] + dz, i0[1] + dy, i0[0] + dx]
    out[inside] = acc
    return out
