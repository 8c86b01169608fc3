"""Temporal correspondence tracking (Strategy 1 of the paper, Sec. 3.3, Eq. 1).

The template's vertices are carried forward through a varying-topology
sequence {(V_t, F_t)}: the tracked points of frame t + 1 are the closest points
on mesh t + 1 of the tracked points of frame t (a BVH built over mesh t + 1, the
closest-point query with the tracked points as queries).  To limit drift, every
`every` frames the tracked points are re-anchored to the template: w_track of
the tracked motion blended with 1 - w_track of the direct template projection
(Eq. 2, the template's own vertices projected onto that mesh); the paper uses
every = 50 and w_track = 0.8.  The track starts from the template vertices;
NearestSurface is the single closest point (k = 1) or, with k > 1, the k-NN
weighted projection (mg_knn_surface_query); the blend is used as it is.
Every step runs in the library's kernels (build, query, blend).
"""

import torch

from . import api


class Tracker:
    """Device-resident tracking state over a sequence of meshes of varying size.

    template_verts [3][N] float32.  max_faces bounds the faces of any frame (one
    BVH buffer and workspace serve every frame).  query: traversal options.
    """

    def __init__(self, template_verts, max_faces, *, every=50, w_track=0.8, query=None, k=1, eps=0.0):
        dev = template_verts.device
        self.template = template_verts
        self.every, self.w_track = int(every), float(w_track)
        self.k, self.eps = int(k), float(eps)
        self.query = dict(query or {})
        self.buf = torch.empty(api.lbvh_bytes(max_faces), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(max(api.lbvh_workspace_bytes(max_faces), 1), dtype=torch.uint8, device=dev)
        n = template_verts.shape[1]
        self.rec = api._query_out(n, dev, True, False, False, False)
        self.anchor = api._query_out(n, dev, True, False, False, False)
        if self.k > 1:
            self.knn = {"face": torch.empty(self.k, n, dtype=torch.int32, device=dev),
                        "dist2": torch.empty(self.k, n, device=dev)}
            self.knn_anchor = dict(self.knn, point=self.anchor["point"])

    def _project(self, bvh, verts, points, out_rec, knn_out):
        if self.k > 1:
            api.knn_surface_query(bvh, verts, points, k=self.k, eps=self.eps, out=knn_out)
        else:
            api.closest_point_query(bvh, verts, points, point=True, bary=False, dist2=False, out=out_rec,
                                    **self.query)

    def step(self, points, verts, faces, t, out):
        """Tracked points of frame t (>= 1) on mesh (verts, faces) into out [3][N], from points [3][N]."""
        bvh = api.LBVH(faces.shape[1], api.MG_PRIM_TRIANGLES, verts.device, buf=self.buf, ws=self.ws)
        api.lbvh_build(verts, faces, bvh=bvh)
        self.rec["point"] = out
        self._project(bvh, verts, points, self.rec, dict(self.knn, point=out) if self.k > 1 else None)
        if self.every and t % self.every == 0:
            self._project(bvh, verts, self.template, self.anchor, self.knn_anchor if self.k > 1 else None)
            api.blend(out, self.anchor["point"], self.w_track, 1.0 - self.w_track, out=out)
        return out


def track_correspondences(template_verts, targets, *, every=50, w_track=0.8, query=None, k=1, eps=0.0, out=None):
    """Tracked template vertices of every frame: [T][3][N] (frame 0 = the template).

    targets: list of (verts [3][V_t] float32, faces [3][F_t] int32) device tensors.
    """
    T = len(targets)
    n = template_verts.shape[1]
    out = torch.empty(T, 3, n, device=template_verts.device) if out is None else out
    api.vertex_buffer_update(template_verts.reshape(1, 3, n), 0, out[0])
    tr = Tracker(template_verts, max(f.shape[1] for _, f in targets), every=every, w_track=w_track, query=query,
                 k=k, eps=eps)
    for t in range(1, T):
        tv, tf = targets[t]
        tr.step(out[t - 1], tv, tf, t, out[t])
    return out
