"""The five seeded workloads.

C1 small       icosphere(4): 2,562 V / 5,120 F, 6 Gaussians per face (30,720),
               60 frames of vector sinusoidal displacement, 10,000 queries
               uniform in the rest bounding box.
C2 refit/rebuild  UV sphere (200 x 100): 20,002 V / 40,000 F with a radial shape,
               100,000 area-weighted Gaussians, 200 frames of radial motion,
               50,000 collision particles uniform in the rest box grown by 10%,
               and per frame a varying-topology target: marching tetrahedra of the
               same deformed surface (about 30-60k faces).
C3 batched     6 UV spheres of 5k..50k faces, 20k..300k Gaussians,
               10k..100k queries, 64 frames each.
C4 differentiable  the C2 template vs 100,000 samples of a deformed
               marching-tetrahedra surface, 100,000 Gaussians; finite-difference
               subset: UV sphere (25 x 10) = 500 faces, 1,250 Gaussians, 2,000 targets.
C5 large       UV sphere (1000 x 250): 250,002 V / 500,000 F, 1,000,000 Gaussians,
               1,000,000 queries, 100 frames; per frame a 2x-face rebuild target
               made by splitting every face once.

Seeds: 60644400 + 10 * config + scene (numpy PCG64).  Everything is produced on
the host in float64 and rounded once to float32 (positions) / int32 (indices),
SoA layout: vertices [3][V], faces [3][F], queries [3][Q].
"""

from dataclasses import dataclass, field

import numpy as np

from .meshes import icosphere, uv_sphere
from .deform import RadialShape, RadialMotion, VectorMotion, radial_template, frames_radial, frames_vector
from .mtet import radial_level_set_target, split_faces_target
from .gaussians import draw_binding, sample_surface


def seed_for(config, scene=0):
    return 60644400 + 10 * int(config) + int(scene)


def _soa_v(v):
    return np.ascontiguousarray(v.T.astype(np.float32))


def _soa_f(f):
    return np.ascontiguousarray(f.T.astype(np.int32))


@dataclass
class Scene:
    """One seeded scene: a fixed-topology template, its frames, binding, queries and targets."""
    name: str
    seed: int
    verts0: np.ndarray            # [3][V] float32 rest pose
    faces: np.ndarray             # [3][F] int32
    binding: dict
    queries: np.ndarray           # [3][Q] float32
    n_frames: int
    kind: str                     # "vector" | "radial"
    _xhat: np.ndarray = None
    _v0: np.ndarray = None
    _shape: object = None
    _motion: object = None
    target_cells: int = 0
    target_kind: str = "none"     # "mtet" | "split" | "none"
    extra: dict = field(default_factory=dict)

    @property
    def n_verts(self):
        return self.verts0.shape[1]

    @property
    def n_faces(self):
        return self.faces.shape[1]

    @property
    def n_gauss(self):
        return self.binding["face"].shape[0]

    def frames(self, ts):
        """Frame store [len(ts)][3][V] float32 for integer frame indices ts."""
        ts = [int(t) for t in ts]
        if self.kind == "vector":
            return frames_vector(self._v0, self._motion, ts)
        return frames_radial(self._xhat, self._shape, self._motion, ts)

    def target(self, t):
        """Varying-topology target of frame t as (verts [3][Vt] f32, faces [3][Ft] i32)."""
        if self.target_kind == "mtet":
            v, f = radial_level_set_target(self._shape, self._motion, float(t), self.target_cells)
        elif self.target_kind == "split":
            vt = self.frames([t])[0].T.astype(np.float64)
            rng = np.random.default_rng([self.seed, int(t)])
            v, f = split_faces_target(vt, self.faces.T.astype(np.int64), rng)
        else:
            raise ValueError(f"scene {self.name} has no varying-topology target")
        return _soa_v(v), _soa_f(f)


def _radial_scene(name, seed, n_lon, n_rings, n_gauss, n_queries, n_frames, grow=0.0,
                  target_kind="none", target_cells=0):
    rng = np.random.default_rng(seed)
    xhat, f = uv_sphere(n_lon, n_rings)
    shape = RadialShape(rng)
    v0 = radial_template(xhat, shape)
    binding = draw_binding(rng, v0, f, n_gauss=n_gauss)
    motion = RadialMotion(rng, n_frames)
    lo, hi = v0.min(0), v0.max(0)
    pad = grow * (hi - lo) / 2.0
    q = rng.uniform(lo - pad, hi + pad, size=(n_queries, 3))
    return Scene(name, seed, _soa_v(v0), _soa_f(f), binding, _soa_v(q), n_frames, "radial",
                 _xhat=xhat, _v0=v0, _shape=shape, _motion=motion,
                 target_kind=target_kind, target_cells=target_cells)


# Grid resolution for the C2 / C4 marching-tetrahedra targets, chosen so that
# each target lands in the 30-60k face range.
MT_CELLS = 58

C3_SCENES = [  # (n_lon, n_rings, gaussians, queries) -> 5k..50k faces
    (100, 25, 20_000, 10_000),
    (100, 50, 50_000, 20_000),
    (200, 50, 100_000, 40_000),
    (300, 50, 150_000, 60_000),
    (200, 100, 200_000, 80_000),
    (250, 100, 300_000, 100_000),
]


def make_config(cfg, scene=0, small=False):
    """Build scene `scene` of workload `cfg` (1..5).

    small=True keeps the structure but shrinks counts (for fast CPU tests).
    """
    cfg = int(cfg)
    seed = seed_for(cfg, scene)
    if cfg == 1:
        rng = np.random.default_rng(seed)
        v0, f = icosphere(2 if small else 4)
        binding = draw_binding(rng, v0, f, per_face=6)
        motion = VectorMotion(rng, 60)
        lo, hi = v0.min(0), v0.max(0)
        q = rng.uniform(lo, hi, size=(500 if small else 10_000, 3))
        return Scene("c1", seed, _soa_v(v0), _soa_f(f), binding, _soa_v(q), 60, "vector",
                     _v0=v0, _motion=motion)
    if cfg == 2:
        if small:
            return _radial_scene("c2s", seed, 40, 20, 8_000, 2_000, 200, grow=0.1,
                                 target_kind="mtet", target_cells=24)
        return _radial_scene("c2", seed, 200, 100, 100_000, 50_000, 200, grow=0.1,
                             target_kind="mtet", target_cells=MT_CELLS)
    if cfg == 3:
        n_lon, n_rings, g, nq = C3_SCENES[scene]
        if small:
            n_lon, n_rings, g, nq = max(8, n_lon // 10), max(4, n_rings // 5), g // 50, nq // 50
        return _radial_scene(f"c3s{scene}", seed, n_lon, n_rings, g, nq, 64)
    if cfg == 4:
        if small:  # the finite-difference subset
            sc = _radial_scene("c4fd", seed, 25, 10, 1_250, 0, 200, target_kind="mtet", target_cells=20)
            n_t = 2_000
        else:
            sc = _radial_scene("c4", seed, 200, 100, 100_000, 0, 200, target_kind="mtet",
                               target_cells=MT_CELLS)
            n_t = 100_000
        rng = np.random.default_rng([seed, 4])
        tv, tf = radial_level_set_target(sc._shape, sc._motion, 0.37 * sc.n_frames, sc.target_cells)
        sc.extra["targets"] = sample_surface(rng, tv, tf, n_t)
        return sc
    if cfg == 5:
        if small:
            return _radial_scene("c5s", seed, 100, 25, 10_000, 10_000, 100, target_kind="split")
        return _radial_scene("c5", seed, 1000, 250, 1_000_000, 1_000_000, 100, target_kind="split")
    raise ValueError(f"unknown workload {cfg}")


CONFIGS = {
    1: "small: icosphere 2,562 V / 5,120 F, 30,720 Gaussians, 60 frames, 10,000 queries",
    2: "refit vs rebuild: 20,002 V / 40,000 F, 100,000 Gaussians, 200 frames, 50,000 particles, MT targets",
    3: "batched: 6 scenes 5k..50k F, 20k..300k Gaussians, 10k..100k queries, 64 frames",
    4: "differentiable: 40,000 F template, 100,000 Gaussians, 100,000 target samples",
    5: "large: 250,002 V / 500,000 F, 1,000,000 Gaussians, 1,000,000 queries, 100 frames",
}
