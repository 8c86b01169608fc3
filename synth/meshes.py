"""Template meshes: geodesic icosphere and UV sphere (AoS, float64 / int64)."""

import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level):
    """Icosahedron subdivided `level` times at edge midpoints, on the unit sphere.

    level 4 gives 2,562 vertices and 5,120 faces.  Faces wind counter-clockwise
    seen from outside.
    """
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        key = e[:, 0] * (nv + 1) + e[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        a = uniq // (nv + 1)
        b = uniq % (nv + 1)
        mid = 0.5 * (v[a] + v[b])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = nv + inv.reshape(3, -1)          # m[0]: edge 01, m[1]: 12, m[2]: 20
        m01, m12, m20 = m[0], m[1], m[2]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1),
        ])
        v = np.concatenate([v, mid])
    return v, f


def uv_sphere(n_lon, n_rings):
    """Latitude/longitude sphere: n_lon * n_rings + 2 vertices, 2 * n_lon * n_rings faces.

    Vertex 0 is the north pole, the last vertex the south pole; ring r (0-based,
    from the north) holds n_lon vertices at polar angle pi * (r + 1) / (n_rings + 1).
    Faces wind counter-clockwise seen from outside.
    """
    if n_lon < 3 or n_rings < 1:
        raise ValueError("uv_sphere needs n_lon >= 3 and n_rings >= 1")
    theta = np.pi * (np.arange(n_rings) + 1) / (n_rings + 1)
    phi = 2.0 * np.pi * np.arange(n_lon) / n_lon
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    ring = np.stack([st * np.cos(phi), st * np.sin(phi), np.broadcast_to(ct, (n_rings, n_lon))], -1)
    v = np.concatenate([[[0.0, 0.0, 1.0]], ring.reshape(-1, 3), [[0.0, 0.0, -1.0]]])
    south = n_lon * n_rings + 1
    j = np.arange(n_lon)
    jn = (j + 1) % n_lon
    top = np.stack([np.zeros(n_lon, np.int64), 1 + j, 1 + jn], 1)
    faces = [top]
    for r in range(n_rings - 1):
        a = 1 + r * n_lon + j
        b = 1 + r * n_lon + jn
        c = 1 + (r + 1) * n_lon + j
        d = 1 + (r + 1) * n_lon + jn
        faces.append(np.stack([a, c, d], 1))
        faces.append(np.stack([a, d, b], 1))
    last = 1 + (n_rings - 1) * n_lon
    bot = np.stack([last + j, np.full(n_lon, south, np.int64), last + jn], 1)
    faces.append(bot)
    return v, np.concatenate(faces).astype(np.int64)


def mesh_aabb(v):
    """Axis-aligned bounds (lo, hi) of an AoS vertex array."""
    return v.min(axis=0), v.max(axis=0)


def triangle_areas(v, f):
    """Triangle areas, used only to weight random draws over faces."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
