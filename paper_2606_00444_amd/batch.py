"""Binding of the batched form (mg_batch_plan_init / mg_batch_run): argument marshalling only.

Every scene-frame's outputs live in per-frame blocks of tensors allocated here
with torch; the work itself is one reset kernel plus one persistent kernel.
"""

import ctypes

import torch

from . import _lib
from .api import _call, _ptr, _stream, lbvh_build


class BatchPlan:
    """All scenes x frames of re-pose, refit and closest-point queries in one launch.

    scenes: list of dicts with device tensors
      frames [T][3][V] float32, faces [3][F] int32, gface [G] int32, bary [2][G],
      q_local [4][G], log_scale [3][G], queries [3][Q] float32,
      and optionally bvh (a triangle LBVH over the faces; built from frame 0 if absent)
      and this scene's traversal: batch (queries per wave), seed, query_tile.
    Options: the plan-wide defaults of batch, seed and query_tile, and
    gauss_tile.  autotune.tune_batch chooses all of them.  After run(), out[i]
    holds scene i's per-frame outputs.
    """

    def __init__(self, scenes, *, batch=4, seed=True, gauss_tile=2048, query_tile=256, normals=True):
        self.scenes = scenes
        self.out = []
        arr = (_lib.BatchScene * len(scenes))()
        for i, sc in enumerate(scenes):
            fr = sc["frames"]
            T, _, V = fr.shape
            F = sc["faces"].shape[1]
            G = sc["gface"].shape[0]
            Q = sc["queries"].shape[1]
            dev = fr.device
            bvh = sc.get("bvh") or lbvh_build(fr[0].contiguous(), sc["faces"])
            sc["bvh"] = bvh
            o = {
                "nodes": torch.empty(T, max(F - 1, 0) * 24, device=dev),
                "roots": torch.empty(T, 8, device=dev),
                "mean": torch.empty(T, 3, G, device=dev), "quat": torch.empty(T, 4, G, device=dev),
                "cov": torch.empty(T, 6, G, device=dev),
                "face": torch.empty(T, Q, dtype=torch.int32, device=dev), "point": torch.empty(T, 3, Q, device=dev),
                "bary": torch.empty(T, 2, Q, device=dev), "dist2": torch.empty(T, Q, device=dev),
                "normal": torch.empty(T, 3, Q, device=dev) if normals else None,
            }
            self.out.append(o)
            s = arr[i]
            s.frames, s.n_frames, s.n_verts = _ptr(fr), T, V
            s.faces, s.n_faces, s.n_gauss = _ptr(sc["faces"]), F, G
            s.gface, s.bary, s.q_local, s.log_scale = (_ptr(sc[k]) for k in ("gface", "bary", "q_local", "log_scale"))
            s.queries, s.n_queries = _ptr(sc["queries"]), Q
            s.bvh, s.bvh_bytes = _ptr(bvh.buf), bvh.nbytes
            s.nodes, s.roots, s.mean, s.quat, s.cov = (_ptr(o[k]) for k in ("nodes", "roots", "mean", "quat", "cov"))
            s.face, s.point, s.qbary, s.dist2, s.normal = (_ptr(o[k]) for k in ("face", "point", "bary", "dist2", "normal"))
        self._arr = arr
        size = ctypes.c_size_t()
        _call("mg_batch_plan_size", ctypes.byref(arr), len(scenes), ctypes.byref(size))
        self.plan = torch.empty(size.value, dtype=torch.uint8, device=scenes[0]["frames"].device)
        self.configure(batch=batch, seed=seed, gauss_tile=gauss_tile, query_tile=query_tile)
        st = ctypes.c_void_p()
        _call("mg_batch_status_word", _ptr(self.plan), ctypes.byref(st))
        self._status_off = st.value - self.plan.data_ptr()

    def configure(self, *, batch=4, seed=True, gauss_tile=2048, query_tile=256, per_scene=None):
        """(Re)write the device plan with new plan-wide defaults and, optionally,
        per-scene traversal overrides per_scene[i] = {batch, seed, query_tile}
        (synchronises the stream; outputs and plan buffer are reused)."""
        arr = self._arr
        for i, sc in enumerate(self.scenes):
            o = dict(sc)
            if per_scene is not None:
                o.update(per_scene[i])
            arr[i].batch = int(o.get("batch") or 0)
            arr[i].seed = -1 if o.get("seed") is None else int(bool(o["seed"]))
            arr[i].query_tile = int(o.get("query_tile") or 0)
        opt = _lib.BatchOptions()
        opt.batch, opt.seed, opt.gauss_tile, opt.query_tile = int(batch), int(bool(seed)), int(gauss_tile), int(query_tile)
        self.options = {"batch": batch, "seed": seed, "gauss_tile": gauss_tile, "query_tile": query_tile,
                        "per_scene": per_scene}
        _call("mg_batch_plan_init", ctypes.byref(arr), len(self.scenes), ctypes.byref(opt), _ptr(self.plan),
              self.plan.numel(), _stream())

    def run(self):
        """Enqueue one run over every scene-frame on torch's current stream."""
        _call("mg_batch_run", _ptr(self.plan), self.plan.numel(), _stream())

    def status(self):
        """The plan's error word after the last run (synchronises)."""
        return int(self.plan[self._status_off:self._status_off + 4].view(torch.int32).item())
