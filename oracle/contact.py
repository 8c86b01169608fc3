"""Sphere-mesh contact step from on-demand normals (collision response), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's simulation drops rigid spheres on the reconstructed mesh and
queries collisions against it every step, recomputing face normals on demand
(Sec. 3.4 step 3, Sec. 4.1); the engine it uses is not part of this work.
Reading for a minimal contact step of spheres of radius r (position x,
velocity v, per step dt under gravity g):

1. semi-implicit Euler: v <- v + g dt, x <- x + v dt;
2. closest point c on the mesh and the unit normal n of its face;
3. side = (x - c) . n; a sphere is in contact when side < 0 (its centre went
   through the surface) or |x - c| < r;
4. contact normal: nh = (x - c) / |x - c| when side >= 0 and |x - c| > 0,
   else n (the face normal; a degenerate face gives no contact);
5. response: x <- c + r nh; if v . nh < 0: v <- v - (1 + e) (v . nh) nh
   (restitution e in [0, 1]).
"""

import numpy as np

from .closest import closest_point_mesh


def step(x, v, verts, faces, dt, g, radius, restitution):
    """One contact step for spheres x, v [3][P]; returns new (x, v, contact [P] bool)."""
    x = np.asarray(x, dtype=np.float64) + 0.0
    v = np.asarray(v, dtype=np.float64) + np.asarray(g, dtype=np.float64)[:, None] * dt
    x = x + v * dt
    r = closest_point_mesh(verts, faces, x)
    c, n = r["point"], r["normal"]
    d = x - c
    dist = np.sqrt((d * d).sum(0))
    side = (d * n).sum(0)
    has_face = (r["face"] >= 0) & ((n * n).sum(0) > 0)
    contact = has_face & ((side < 0) | (dist < radius))
    use_d = (side >= 0) & (dist > 0)
    nh = np.where(use_d, d / np.where(dist > 0, dist, 1.0), n)
    x = np.where(contact, c + radius * nh, x)
    vn = (v * nh).sum(0)
    hit = contact & (vn < 0)
    v = np.where(hit, v - (1.0 + restitution) * vn * nh, v)
    return x, v, contact

