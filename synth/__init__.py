"""Seeded synthetic inputs for the dynamic mesh-Gaussian update.

This package only *draws* inputs: template meshes, per-frame vertex
positions, varying-topology targets, face-bound Gaussian bindings and query
points.  It contains none of the method's arithmetic (no triangle frames,
no re-posing, no Morton codes, no BVH, no closest points); both the oracle
and the HIP path read the arrays it produces.

The paper evaluates on six captured dynamic scenes of 200 frames each with
meshes of 10^3-10^4 vertices (Sec. 3.4, Sec. 4).  That dataset is not
available here; these generators stand in for it with smooth, seeded
deformations of sphere-like templates of the sizes the workloads name.
"""

from .meshes import icosphere, uv_sphere, mesh_aabb, triangle_areas
from .deform import (RadialShape, RadialMotion, VectorMotion, radial_template,
                     frames_radial, frames_vector)
from .mtet import marching_tetrahedra, radial_level_set_target, split_faces_target
from .gaussians import draw_binding, sample_surface
from .configs import (CONFIGS, make_config, Scene, seed_for)

__all__ = [
    "icosphere", "uv_sphere", "mesh_aabb", "triangle_areas",
    "RadialShape", "RadialMotion", "VectorMotion", "radial_template",
    "frames_radial", "frames_vector",
    "marching_tetrahedra", "radial_level_set_target", "split_faces_target",
    "draw_binding", "sample_surface",
    "CONFIGS", "make_config", "Scene", "seed_for",
]
