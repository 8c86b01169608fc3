"""Temporal correspondence tracking (Strategy 1, Sec. 3.3, Eq. 1), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The template's vertices are carried forward through a varying-topology
sequence: the tracked points of frame t+1 are the closest points on mesh t+1 of
the tracked points of frame t.  To limit drift, every `every` frames the
tracked points are re-anchored to the template: 80% tracked motion blended with
20% direct template projection (the projection of the template's own vertices
onto that frame's mesh, Eq. 2).

Readings (the paper is silent on these): the track starts from the template
vertices at frame 0; NearestSurface is the single closest point (k = 1, as in
closest.py), or optionally the k-NN weighted projection (knn.py); a
re-anchoring frame is one whose index is a positive multiple of
`every`, and the blend is used as it is (not projected again).
"""

import numpy as np

from .closest import closest_point_mesh
from .knn import knn_surface


def track_step(points, verts, faces, k=1, eps=0.0):
    """Eq. 1 for one frame: NearestSurface on (verts, faces) of every point [3][N]
    (the closest point for k = 1, else the k-NN weighted projection of knn.py)."""
    if k <= 1:
        return closest_point_mesh(verts, faces, points)["point"]
    return knn_surface(verts, faces, points, k=k, eps=eps)["point"]


def track(template_verts, targets, every=50, w_track=0.8, start=None, k=1, eps=0.0):
    """Tracked vertices of every frame of `targets` (a list of (verts [3][V_t], faces [3][F_t])).

    Returns [T][3][N]: frame 0 is the start (the template vertices unless
    `start` is given), frame t >= 1 the tracked points on targets[t].
    """
    V0 = np.asarray(template_verts, dtype=np.float64)
    cur = V0.copy() if start is None else np.asarray(start, dtype=np.float64).copy()
    out = [cur.copy()]
    for t in range(1, len(targets)):
        tv, tf = targets[t]
        nxt = track_step(cur, tv, tf, k, eps)
        if every and t % every == 0:
            anchor = track_step(V0, tv, tf, k, eps)
            nxt = w_track * nxt + (1.0 - w_track) * anchor
        out.append(nxt)
        cur = nxt
    return np.stack(out)
