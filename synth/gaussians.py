"""Seeded face-bound Gaussian bindings and surface samples.

A binding is the per-Gaussian tuple (face id, barycentric (b1, b2), local unit
quaternion (w, x, y, z), log-scales (3)).  Faces are drawn either a fixed number
per face or area-weighted; the result is sorted by face with CSR offsets.
Barycentrics are uniform on the triangle (Osada et al. 2002:
(1 - sqrt r1, sqrt r1 (1 - r2), sqrt r1 r2)); local rotations are uniform on
SO(3) (Shoemake 1992) with w >= 0; log-scales are i.i.d. normal.
"""

import numpy as np

from .meshes import triangle_areas


def _uniform_bary(rng, n):
    r1 = rng.random(n)
    r2 = rng.random(n)
    s = np.sqrt(r1)
    return np.stack([s * (1.0 - r2), s * r2])            # (b1, b2)


def _uniform_quat(rng, n):
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)])   # (w, x, y, z)
    q[:, q[0] < 0] *= -1.0
    return q


def draw_binding(rng, v, f, n_gauss=None, per_face=None, log_scale_mean=-4.0, log_scale_std=0.3):
    """Draw a face-sorted binding on mesh (v, f) (AoS).

    Exactly one of n_gauss (area-weighted multinomial over faces) or per_face
    (that many per face, face-major) must be given.  Returns a dict of
    SoA float32 / int32 arrays: face [G], face_offsets [F+1], bary [2][G],
    q_local [4][G], log_scale [3][G].
    """
    nf = f.shape[0]
    if per_face is not None:
        counts = np.full(nf, int(per_face), np.int64)
    else:
        area = triangle_areas(v, f)
        counts = rng.multinomial(int(n_gauss), area / area.sum())
    face = np.repeat(np.arange(nf, dtype=np.int64), counts)
    g = face.size
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    bary = _uniform_bary(rng, g)
    q = _uniform_quat(rng, g)
    ls = rng.normal(log_scale_mean, log_scale_std, size=(3, g))
    return {
        "face": face.astype(np.int32),
        "face_offsets": offsets,
        "bary": bary.astype(np.float32),
        "q_local": q.astype(np.float32),
        "log_scale": ls.astype(np.float32),
    }


def sample_surface(rng, v, f, n):
    """n points area-uniform on mesh (v, f) (AoS), returned SoA float32 [3][n]."""
    area = triangle_areas(v, f)
    fid = rng.choice(f.shape[0], size=n, p=area / area.sum())
    b = _uniform_bary(rng, n)
    a, bb, c = v[f[fid, 0]], v[f[fid, 1]], v[f[fid, 2]]
    p = (1.0 - b[0] - b[1])[:, None] * a + b[0][:, None] * bb + b[1][:, None] * c
    return p.T.astype(np.float32)
