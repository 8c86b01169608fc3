"""Index signed-distance grid: the SDF the paper builds from the template faces
beside the BVH (Sec. 3.4, Initialization: structures storing only indices, so
they serve every frame).

At construction every grid node stores the ids of its k nearest template faces
(the k-NN query of the library on the node positions); update(verts) then
recomputes every node's signed distance from those faces' current vertices in
one pass over the grid (mg_sdf_update), and sample(queries) interpolates it
trilinearly (mg_sdf_sample).  See include/mgu.h for the exact definition.
"""

import torch

from . import api
from .api import _call, _ptr, _f32, _i32, _stream


class IndexSDF:
    """Grid over [lo, lo + h (dims - 1)] with the k nearest template faces per node.

    template_verts [3][V] float32 and faces [3][F] int32 on one device; lo a
    3-tuple, h > 0, dims = (nx, ny, nz) each >= 2.
    """

    def __init__(self, template_verts, faces, lo, h, dims, k=4):
        self.faces, self.lo, self.h, self.dims, self.k = faces, tuple(float(x) for x in lo), float(h), tuple(
            int(d) for d in dims), int(k)
        dev = template_verts.device
        n = self.dims[0] * self.dims[1] * self.dims[2]
        self.n_nodes = n
        self.points = torch.empty(3, n, device=dev)
        _call("mg_grid_points", *self.lo, self.h, *self.dims, _ptr(self.points), _stream())
        bvh = api.lbvh_build(template_verts, faces)
        r = api.knn_surface_query(bvh, template_verts, self.points, k=self.k, out={"point": None})
        self.face_k = r["face"]                   # [k][n] int32: the indices kept across frames
        self.sdf = torch.empty(n, device=dev)
        self.face = torch.empty(n, dtype=torch.int32, device=dev)

    def update(self, verts):
        """Signed distances of every node for the vertex positions verts [3][V] (into self.sdf)."""
        _call("mg_sdf_update", _ptr(_f32(verts, 3, "verts")), verts.shape[1], _ptr(_i32(self.faces)),
              self.faces.shape[1], _ptr(self.face_k), self.k, *self.lo, self.h, *self.dims, _ptr(self.sdf),
              _ptr(self.face), _stream())
        return self.sdf

    def sample(self, queries, out=None):
        """Trilinear interpolation of the grid at queries [3][Q] (+inf outside the grid)."""
        nq = _f32(queries, 3, "queries").shape[1]
        out = torch.empty(nq, device=queries.device) if out is None else out
        _call("mg_sdf_sample", _ptr(self.sdf), *self.lo, self.h, *self.dims, _ptr(queries), nq, _ptr(_f32(out)),
              _stream())
        return out
