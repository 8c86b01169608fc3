"""Sphere-mesh contact step from on-demand face normals (collision response).

Spheres of one radius fall under gravity onto the mesh and bounce off it: each
step integrates them (mg_particles_integrate), finds the closest point, face and
face normal of every sphere centre on the current mesh through the refit BVH
(mg_closest_point_query), and resolves contacts (mg_contact_response).  The
definition is in include/mgu.h.
"""

import torch

from . import api
from .api import _call, _ptr, _f32, _stream


class Spheres:
    """x, v [3][n] float32 device tensors (updated in place); radius, restitution in [0, 1]."""

    def __init__(self, x, v, radius, restitution=0.5, gravity=(0.0, 0.0, -9.8), query=None):
        self.x, self.v = _f32(x, 3, "x"), _f32(v, 3, "v")
        self.radius, self.restitution, self.gravity = float(radius), float(restitution), tuple(map(float, gravity))
        n = x.shape[1]
        self.rec = api._query_out(n, x.device, True, False, False, True)
        self.rec["face"].fill_(-1)              # no previous step: no hints
        self.contact = torch.empty(n, dtype=torch.int32, device=x.device)
        self.query = dict(query or {})

    def step(self, bvh, verts, dt):
        """One step against the mesh of bvh (refit to verts by the caller).  Each
        sphere's closest-point query starts from its face of the previous step."""
        n = self.x.shape[1]
        _call("mg_particles_integrate", _ptr(self.x), _ptr(self.v), n, *self.gravity, float(dt), _stream())
        api.closest_point_query(bvh, verts, self.x, normal=True, out=self.rec, hint=self.rec["face"], **self.query)
        _call("mg_contact_response", _ptr(self.x), _ptr(self.v), n, _ptr(self.rec["point"]),
              _ptr(self.rec["normal"]), _ptr(self.rec["face"]), self.radius, self.restitution, _ptr(self.contact),
              _stream())
        return self.contact
