"""30-bit Morton codes defined in IEEE binary32, and the stable sort.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper builds its collision acceleration structure once from the template
faces (Sec. 3.4, Initialization) but does not say which BVH.  The reading is a
linear BVH (Karras 2012) over face centroids.  So that "bit-exact Morton codes"
means something between a float64 oracle and a float32 device, the code is
defined entirely in binary32 with round-to-nearest-even after every operation
and no fused multiply-add:

  s      = (v0 + v1) + v2 per axis (three times the centroid); for point
           primitives s = p
  lo, hi = min, max of s over all primitives (per axis; exact)
  scale  = 1024 / (hi - lo) if hi > lo else 0
  q      = min(1023, trunc((s - lo) * scale))
  code   = spread(qx) << 2 | spread(qy) << 1 | spread(qz), spread putting bit i at bit 3 i.

numpy float32 array arithmetic rounds every operation to binary32 and never
contracts, which is exactly this definition.
"""

import numpy as np


def centroid_sums(verts, faces):
    """s [3][n] float32: (v0 + v1) + v2 per axis, or the points themselves if faces is None."""
    V = np.asarray(verts, dtype=np.float32)
    if faces is None:
        return V.copy()
    F = np.asarray(faces).astype(np.int64)
    return (V[:, F[0]] + V[:, F[1]]) + V[:, F[2]]


def quantize(s):
    """Per-axis 10-bit cells q [3][n] uint32, plus lo [3], scale [3] (float32)."""
    s = np.asarray(s, dtype=np.float32)
    n = s.shape[1]
    if n == 0:
        return np.zeros((3, 0), np.uint32), np.zeros(3, np.float32), np.zeros(3, np.float32)
    lo = s.min(axis=1)
    hi = s.max(axis=1)
    ext = hi - lo
    safe = np.where(ext > 0, ext, np.float32(1.0)).astype(np.float32)
    scale = np.where(hi > lo, np.float32(1024.0) / safe, np.float32(0.0)).astype(np.float32)
    x = (s - lo[:, None]) * scale[:, None]
    q = np.minimum(x.astype(np.uint32), np.uint32(1023))
    return q, lo, scale


def spread10(q):
    """Put bit i of a 10-bit integer at bit 3 i (plain bit loop)."""
    q = np.asarray(q, dtype=np.uint32)
    out = np.zeros_like(q)
    for i in range(10):
        out |= ((q >> np.uint32(i)) & np.uint32(1)) << np.uint32(3 * i)
    return out


def morton_codes(verts, faces):
    """uint32 [n] codes of the primitives (faces, or points if faces is None)."""
    q, _, _ = quantize(centroid_sums(verts, faces))
    return (spread10(q[0]) << np.uint32(2)) | (spread10(q[1]) << np.uint32(1)) | spread10(q[2])


def sort_codes(codes):
    """Stable ascending sort: (sorted codes, perm) with perm[leaf] = original primitive id.

    Sorting by code with a stable sort from index order is the same as sorting
    the pairs (code, id), so the permutation is unique.
    """
    codes = np.asarray(codes, dtype=np.uint32)
    perm = np.argsort(codes, kind="stable")
    return codes[perm], perm.astype(np.int32)


def quantize_fp64(verts, faces):
    """The same cells computed in float64 (reported as boundary ties where they differ)."""
    V = np.asarray(verts, dtype=np.float64)
    if faces is None:
        s = V
    else:
        F = np.asarray(faces).astype(np.int64)
        s = V[:, F[0]] + V[:, F[1]] + V[:, F[2]]
    lo, hi = s.min(axis=1), s.max(axis=1)
    scale = np.where(hi > lo, 1024.0 / np.where(hi > lo, hi - lo, 1.0), 0.0)
    return np.minimum(np.floor((s - lo[:, None]) * scale[:, None]), 1023).astype(np.uint32)
