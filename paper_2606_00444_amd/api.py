"""Thin PyTorch binding over libmgu's C ABI (argument marshalling only).

Every function takes contiguous device tensors, passes their pointers and
torch's current HIP stream to the library, and returns tensors it allocated
with torch (torch owns device memory; the library never allocates).  All
arithmetic happens in the HIP kernels; nothing here computes on the host.
"""

import ctypes
import math

import torch

from . import _lib
from ._lib import MG_PRIM_POINTS, MG_PRIM_TRIANGLES, MG_QUERY_AUTO, MG_QUERY_BATCH, MG_QUERY_LANE, LbvhLayout, QueryOptions

__all__ = [
    "frame_index", "vertex_buffer_update", "fill", "blend", "mesh_gaussian_update", "mesh_gaussian_update_backward",
    "LBVH", "query_order", "lbvh_bytes", "lbvh_workspace_bytes", "lbvh_build", "lbvh_build_static", "frame_update", "lbvh_refit", "closest_point_query", "closest_point_bruteforce",
    "nearest_point_query", "knn_surface_query", "mean", "chamfer", "point_mesh_backward", "chamfer_backward", "adam_step",
    "validate_indices", "validate_finite", "version", "check_device",
]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, shape0=None, name="tensor"):
    if t is None:
        return None
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if shape0 is not None and (t.dim() != 2 or t.shape[0] != shape0):
        raise ValueError(f"{name} must be [{shape0}][n], got {tuple(t.shape)}")
    return t


def _i32(t, name="tensor"):
    if t is None:
        return None
    if t.dtype != torch.int32:
        raise TypeError(f"{name} must be int32")
    return t


def _f64(t, name="tensor"):
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return t


def _call(name, *args):
    lib = _lib.load()
    _lib.check(name, getattr(lib, name)(*args))


def version():
    return _lib.load().mg_version()


def check_device():
    _call("mg_check_device")


def frame_index(step, f_recon_num, f_recon_den, f_sim, n_frames):
    """k = min(floor(step * f_recon / f_sim), n_frames - 1) in integer arithmetic."""
    k = ctypes.c_int32()
    _call("mg_frame_index", step, f_recon_num, f_recon_den, f_sim, n_frames, ctypes.byref(k))
    return k.value


def vertex_buffer_update(frames, k, live):
    """live[3][V] <- frames[k] of a [T][3][V] float32 frame store (device copy)."""
    _f32(frames, name="frames")
    T, three, V = frames.shape
    if three != 3 or tuple(live.shape) != (3, V):
        raise ValueError("frames must be [T][3][V] and live [3][V]")
    _call("mg_vertex_buffer_update", _ptr(frames), T, V, int(k), _ptr(_f32(live, 3, "live")), _stream())
    return live


def fill(x, value=0.0):
    """x[:] = value on the device (float32, contiguous); graph-capturable."""
    _call("mg_fill", _ptr(_f32(x)), x.numel(), float(value), _stream())
    return x


def blend(a, b, wa, wb, out=None):
    """out = wa * a + wb * b on the device (float32, same shape; out may be a or b)."""
    if a.shape != b.shape:
        raise ValueError("blend: a and b must have the same shape")
    out = torch.empty_like(a) if out is None else out
    if out.shape != a.shape:
        raise ValueError("blend: out must have the shape of a")
    _call("mg_blend", _ptr(_f32(a)), _ptr(_f32(b)), float(wa), float(wb), _ptr(_f32(out)), a.numel(), _stream())
    return out


def mesh_gaussian_update(verts, faces, gface, bary, q_local, log_scale, offset=None, *, out=None,
                         quat=True, cov=True, rot=False):
    """Re-pose face-bound Gaussians; returns dict of mean [3][G], quat [4][G], cov [6][G], rot [9][G]."""
    _f32(verts, 3, "verts"); _i32(faces, "faces"); _i32(gface, "gface")
    _f32(bary, 2, "bary"); _f32(q_local, 4, "q_local"); _f32(log_scale, 3, "log_scale"); _f32(offset, None, "offset")
    G = gface.shape[0]
    dev = verts.device
    out = dict(out or {})
    if "mean" not in out:
        out["mean"] = torch.empty(3, G, device=dev)
    if quat and "quat" not in out:
        out["quat"] = torch.empty(4, G, device=dev)
    if cov and "cov" not in out:
        out["cov"] = torch.empty(6, G, device=dev)
    if rot and "rot" not in out:
        out["rot"] = torch.empty(9, G, device=dev)
    _call("mg_mesh_gaussian_update", _ptr(verts), verts.shape[1], _ptr(faces), faces.shape[1], _ptr(gface),
          _ptr(bary), _ptr(q_local), _ptr(log_scale), _ptr(offset), G, 0, _ptr(out["mean"]),
          _ptr(out.get("quat")), _ptr(out.get("cov")), _ptr(out.get("rot")), _stream())
    return out


def mesh_gaussian_update_backward(verts, faces, gface, bary, q_local, log_scale, offset, g_mean,
                                  g_rot=None, g_cov=None, g_verts=None):
    """dL/dV [3][V] (accumulated into g_verts if given) of the re-pose."""
    if g_verts is None:
        g_verts = torch.zeros_like(verts)
    G = gface.shape[0]
    _call("mg_mesh_gaussian_update_backward", _ptr(verts), verts.shape[1], _ptr(faces), faces.shape[1],
          _ptr(gface), _ptr(bary), _ptr(q_local), _ptr(log_scale), _ptr(offset), G, _ptr(_f32(g_mean, 3, "g_mean")),
          _ptr(_f32(g_rot, 9)), _ptr(_f32(g_cov, 6)), _ptr(_f32(g_verts, 3)), _stream())
    return g_verts


def _layout(n, kind):
    L = LbvhLayout()
    _call("mg_lbvh_layout_query", n, kind, ctypes.byref(L))
    return L


def lbvh_workspace_bytes(n_prims, kind=MG_PRIM_TRIANGLES):
    ws = ctypes.c_size_t()
    _call("mg_lbvh_workspace_size", int(n_prims), int(kind), ctypes.byref(ws))
    return ws.value


def lbvh_bytes(n_prims, kind=MG_PRIM_TRIANGLES):
    return _layout(int(n_prims), int(kind)).total_bytes


class LBVH:
    """A linear BVH in one device buffer (layout as documented in include/mgu.h)."""

    def __init__(self, n_prims, kind, device, buf=None, ws=None):
        self.n = int(n_prims)
        self.kind = int(kind)
        self.n_verts = None                 # vertex count of the last build (set by lbvh_build)
        self.layout = _layout(self.n, self.kind)
        need = lbvh_workspace_bytes(self.n, self.kind)
        if buf is None:
            buf = torch.empty(self.layout.total_bytes, dtype=torch.uint8, device=device)
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        if buf.numel() < self.layout.total_bytes or ws.numel() < need:
            raise ValueError("buffer or workspace too small for this BVH")
        self.buf = buf[:self.layout.total_bytes]
        self.ws = ws

    @property
    def nbytes(self):
        return self.layout.total_bytes

    def section(self, name, dtype, count):
        """A typed view of one section of the buffer (no copy)."""
        off = getattr(self.layout, "off_" + name)
        item = torch.empty((), dtype=dtype).element_size()
        return self.buf[off:off + count * item].view(dtype)


def lbvh_build(verts, faces=None, *, bvh=None):
    """Build an LBVH over faces [3][F] of verts, or over the points verts [3][N] if faces is None."""
    _f32(verts, 3, "verts")
    kind = MG_PRIM_POINTS if faces is None else MG_PRIM_TRIANGLES
    n = verts.shape[1] if faces is None else _i32(faces, "faces").shape[1]
    if bvh is None or bvh.n != n or bvh.kind != kind:
        bvh = LBVH(n, kind, verts.device)
    _call("mg_lbvh_build", _ptr(verts), verts.shape[1], _ptr(faces), n, kind, _ptr(bvh.buf), bvh.nbytes,
          _ptr(bvh.ws), bvh.ws.numel(), _stream())
    bvh.n_verts = verts.shape[1]
    return bvh


def lbvh_build_static(verts, faces, bvh):
    """mg_lbvh_build_static: build into the existing bvh (an LBVH of the right size and
    kind) with the library's static sort scratch instead of bvh.ws; at most 2^20
    primitives.  Calls overlapping in time on one device race on that scratch."""
    _f32(verts, 3, "verts")
    kind = MG_PRIM_POINTS if faces is None else MG_PRIM_TRIANGLES
    n = verts.shape[1] if faces is None else _i32(faces, "faces").shape[1]
    if bvh.n != n or bvh.kind != kind:
        raise ValueError("bvh was sized for another primitive count or kind")
    _call("mg_lbvh_build_static", _ptr(verts), verts.shape[1], _ptr(faces), n, kind, _ptr(bvh.buf), bvh.nbytes,
          _stream())
    bvh.n_verts = verts.shape[1]
    return bvh


def _same_verts(bvh, verts, what):
    """Vertex arrays later passed with a BVH must have the build's vertex count: the
    kernels read vertices through the face ids stored at the build, unchecked."""
    _f32(verts, 3, "verts")
    if bvh.n_verts is not None and verts.shape[1] != bvh.n_verts:
        raise ValueError(f"{what}: verts has {verts.shape[1]} vertices, the BVH was built on {bvh.n_verts}")
    return verts


def lbvh_refit(bvh, verts):
    """Recompute every box of bvh for new positions verts (topology unchanged)."""
    _call("mg_lbvh_refit", _ptr(_same_verts(bvh, verts, "lbvh_refit")), verts.shape[1], _ptr(bvh.buf), bvh.nbytes, bvh.n,
          bvh.kind, _stream())
    return bvh


def frame_update(frames, k, live, faces, gface, bary, q_local, log_scale, bvh, offset=None, *, out=None,
                 quat=True, cov=True, rot=False):
    """One launch of the per-frame update: live[3][V] <- frames[k], the Gaussians re-posed
    from frame k (returns the output dict as mesh_gaussian_update), bvh refit on frame k."""
    _f32(frames, name="frames")
    T, three, V = frames.shape
    if three != 3 or tuple(live.shape) != (3, V):
        raise ValueError("frames must be [T][3][V] and live [3][V]")
    _f32(live, 3, "live"); _i32(faces, "faces"); _i32(gface, "gface")
    _f32(bary, 2, "bary"); _f32(q_local, 4, "q_local"); _f32(log_scale, 3, "log_scale"); _f32(offset, None, "offset")
    if bvh.kind != MG_PRIM_TRIANGLES or bvh.n != faces.shape[1]:
        raise ValueError("frame_update: bvh must be a triangle BVH over faces")
    if bvh.n_verts is not None and bvh.n_verts != V:
        raise ValueError(f"frame_update: frames have {V} vertices, the BVH was built on {bvh.n_verts}")
    G = gface.shape[0]
    dev = live.device
    out = dict(out or {})
    if "mean" not in out:
        out["mean"] = torch.empty(3, G, device=dev)
    if quat and "quat" not in out:
        out["quat"] = torch.empty(4, G, device=dev)
    if cov and "cov" not in out:
        out["cov"] = torch.empty(6, G, device=dev)
    if rot and "rot" not in out:
        out["rot"] = torch.empty(9, G, device=dev)
    _call("mg_frame_update", _ptr(frames), T, V, int(k), _ptr(live), _ptr(faces), faces.shape[1], _ptr(gface),
          _ptr(bary), _ptr(q_local), _ptr(log_scale), _ptr(offset), G, _ptr(out["mean"]), _ptr(out.get("quat")),
          _ptr(out.get("cov")), _ptr(out.get("rot")), _ptr(bvh.buf), bvh.nbytes, _stream())
    return out


def _opts(kernel, batch, seed=False, order=None, counters=None, queue=None, hint=None, warm=False, waves=0):
    """ctypes options for the traversal ("auto" | "lane" | "batch"); None when automatic.

    queue: a device int32 [1] work counter for the batch kernel's dynamic
    batch assignment (zeroed by the call itself), or None for static.
    hint: device int32 [Q] original ids to start the queries from, or None.
    warm (chamfer): start from the nearest-neighbour arrays' current contents.
    waves: the batch kernel's register allocation on triangles (0: by launch size, 4 or 5)."""
    auto = kernel in (None, "auto") and not batch and not seed and order is None and counters is None
    if waves not in (0, 4, 5):
        raise ValueError("waves must be 0, 4 or 5")
    if auto and queue is None and hint is None and not warm and not waves:
        return None
    k = {"auto": MG_QUERY_AUTO, None: MG_QUERY_AUTO, "lane": MG_QUERY_LANE, "batch": MG_QUERY_BATCH}[kernel]
    o = QueryOptions()
    o.kernel = k
    o.batch = int(batch or 0)
    o.seed = 1 if auto else int(bool(seed))           # the automatic choice has the seed on
    o.warm = int(bool(warm))
    o.waves = int(waves)
    if queue is not None:
        if queue.dtype != torch.int32 or queue.numel() < 1:
            raise TypeError("queue must be int32 [1]")
        o.queue = _ptr(queue)
    if hint is not None:
        if hint.dtype != torch.int32 or not hint.is_contiguous():
            raise TypeError("hint must be a contiguous int32 tensor")
        o.hint = _ptr(hint)
    if order is not None:
        if order.dtype != torch.int32:
            raise TypeError("order must be int32")
        o.order = _ptr(order)
    if counters is not None:
        if counters.dtype != torch.int64 or counters.numel() < 4:
            raise TypeError("counters must be int64 [4]")
        o.counters = _ptr(counters)
    return ctypes.byref(o)


def query_order(queries):
    """Morton order of query points [3][Q] (int32 permutation), from a point LBVH build."""
    bvh = lbvh_build(_f32(queries, 3, "queries"), None)
    return bvh.section("prim", torch.int32, bvh.n).clone()


def _queue(dynamic, device):
    """A work counter for one traversal call with dynamic batch assignment (its
    own word, so calls on different streams never share one; the call zeroes
    it on its stream), or None."""
    return torch.empty(1, dtype=torch.int32, device=device) if dynamic else None


def _hint(hint, nq):
    """A hint array checked for length (None passes through)."""
    if hint is not None and hint.numel() < nq:
        raise ValueError(f"hint has {hint.numel()} entries for {nq} queries")
    return hint


def _query_out(nq, device, point, bary, dist2, normal):
    return {
        "face": torch.empty(nq, dtype=torch.int32, device=device),
        "point": torch.empty(3, nq, device=device) if point else None,
        "bary": torch.empty(2, nq, device=device) if bary else None,
        "dist2": torch.empty(nq, device=device) if dist2 else None,
        "normal": torch.empty(3, nq, device=device) if normal else None,
    }


def closest_point_query(bvh, verts, queries, max_dist2=math.inf, *, point=True, bary=True, dist2=True,
                        normal=False, out=None, kernel=None, batch=0, seed=False, dynamic=False, order=None,
                        counters=None, hint=None, waves=0):
    """Closest point on the mesh of a triangle LBVH for every query [3][Q].

    kernel: None/"auto", "lane" or "batch" (batch = queries per wave), dynamic:
    batches taken from a work counter instead of dealt statically; hint: int32
    [Q] face ids to start from (e.g. the previous frame's out["face"], which may
    be the very array this call overwrites) - see mg_query_options; waves: the
    batch kernel's register allocation (0: by launch size, 4 or 5).  out: a dict
    of output tensors to fill (face, and point, bary, dist2, normal or None each).
    """
    if bvh.kind != MG_PRIM_TRIANGLES:
        raise ValueError("closest_point_query needs a triangle BVH")
    nq = _f32(queries, 3, "queries").shape[1]
    _same_verts(bvh, verts, "closest_point_query")
    o = out if out is not None else _query_out(nq, queries.device, point, bary, dist2, normal)
    _call("mg_closest_point_query", _ptr(bvh.buf), bvh.nbytes, bvh.n, _ptr(verts), verts.shape[1],
          _ptr(queries), nq, float(max_dist2), _ptr(o["face"]), _ptr(o.get("point")), _ptr(o.get("bary")),
          _ptr(o.get("dist2")), _ptr(o.get("normal")),
          _opts(kernel, batch, seed, order, counters, _queue(dynamic, queries.device), _hint(hint, nq),
                waves=waves), _stream())
    return o


def closest_point_bruteforce(verts, faces, queries, max_dist2=math.inf, *, normal=False):
    """All-faces closest point (self-check path, same contract as closest_point_query)."""
    nq = _f32(queries, 3, "queries").shape[1]
    o = _query_out(nq, queries.device, True, True, True, normal)
    _call("mg_closest_point_bruteforce", _ptr(verts), verts.shape[1], _ptr(_i32(faces)), faces.shape[1],
          _ptr(queries), nq, float(max_dist2), _ptr(o["face"]), _ptr(o["point"]), _ptr(o["bary"]),
          _ptr(o["dist2"]), _ptr(o["normal"]), _stream())
    return o


def knn_surface_query(bvh, verts, queries, k=4, eps=0.0, max_dist2=math.inf, *, out=None, counters=None):
    """k-NN weighted surface projection: dict face [k][Q] int32, dist2 [k][Q], point [3][Q]
    (out={"point": None} skips the weighted point)."""
    if bvh.kind != MG_PRIM_TRIANGLES:
        raise ValueError("knn_surface_query needs a triangle BVH")
    nq = _f32(queries, 3, "queries").shape[1]
    _same_verts(bvh, verts, "knn_surface_query")
    o = dict(out or {})
    for key, shape, dt in (("face", (k, nq), torch.int32), ("dist2", (k, nq), torch.float32), ("point", (3, nq), torch.float32)):
        if key not in o or (o[key] is None and key != "point"):
            o[key] = torch.empty(shape, dtype=dt, device=queries.device)
    _call("mg_knn_surface_query", _ptr(bvh.buf), bvh.nbytes, bvh.n, _ptr(verts), verts.shape[1], _ptr(queries), nq,
          int(k), float(eps), float(max_dist2), _ptr(_i32(o["face"])), _ptr(_f32(o["dist2"])), _ptr(_f32(o["point"])),
          _ptr(counters), _stream())
    return o


def nearest_point_query(bvh, points, queries, max_dist2=math.inf, *, kernel=None, batch=0, seed=False,
                        dynamic=False, order=None, counters=None, hint=None):
    """(index [Q] int32, dist2 [Q]) of the nearest point of a point LBVH."""
    if bvh.kind != MG_PRIM_POINTS:
        raise ValueError("nearest_point_query needs a point BVH")
    nq = _f32(queries, 3, "queries").shape[1]
    if _f32(points, 3, "points").shape[1] != bvh.n:
        raise ValueError(f"nearest_point_query: points has {points.shape[1]} entries, the BVH {bvh.n}")
    idx = torch.empty(nq, dtype=torch.int32, device=queries.device)
    d2 = torch.empty(nq, device=queries.device)
    _call("mg_nearest_point_query", _ptr(bvh.buf), bvh.nbytes, bvh.n, _ptr(points), _ptr(queries), nq,
          float(max_dist2), _ptr(idx), _ptr(d2),
          _opts(kernel, batch, seed, order, counters, _queue(dynamic, queries.device), _hint(hint, nq)), _stream())
    return idx, d2


_reduce_ws = {}


def _rws(device):
    key = str(device)
    if key not in _reduce_ws:
        sz = ctypes.c_size_t()
        _call("mg_reduce_workspace_size", 0, ctypes.byref(sz))
        _reduce_ws[key] = torch.empty(sz.value, dtype=torch.uint8, device=device)
    return _reduce_ws[key]


def mean(x, out=None):
    """Deterministic float64 mean of a float32 device tensor (returns a 1-element float64 tensor)."""
    out = out if out is not None else torch.empty(1, dtype=torch.float64, device=x.device)
    ws = _rws(x.device)
    _call("mg_mean", _ptr(_f32(x)), x.numel(), _ptr(out), _ptr(ws), ws.numel(), _stream())
    return out


def chamfer(a, bvh_a, b, bvh_b, *, out=None, add=None, kernel=None, batch=0, seed=False, warm=False):
    """Two-sided Chamfer: dict nn_ab, d_ab, nn_ba, d_ba and loss [3] (float64: mean d_ab,
    mean d_ba, their sum plus add), with means = loss[0:2] and total = loss[2:3] as views.

    out: optional dict of preallocated outputs with those keys (loss may be any
    contiguous float64 [3] view).  add: an optional float64 device scalar folded
    into the total.  warm: out's nn_ab / nn_ba hold earlier answers (e.g. the
    previous step's; -1 for none) that start the queries."""
    na, nb = _f32(a, 3, "a").shape[1], _f32(b, 3, "b").shape[1]
    dev = a.device
    o = dict(out or {})
    for k, n, dt in (("nn_ab", na, torch.int32), ("d_ab", na, torch.float32), ("nn_ba", nb, torch.int32),
                     ("d_ba", nb, torch.float32), ("loss", 3, torch.float64)):
        if o.get(k) is None:
            o[k] = torch.empty(n, dtype=dt, device=dev)
    if add is not None and (add.dtype != torch.float64 or add.numel() != 1):
        raise TypeError("add must be a float64 device scalar")
    ws = _rws(dev)
    _call("mg_chamfer", _ptr(a), na, _ptr(bvh_a.buf), bvh_a.nbytes, _ptr(b), nb, _ptr(bvh_b.buf),
          bvh_b.nbytes, _ptr(_i32(o["nn_ab"])), _ptr(_f32(o["d_ab"])), _ptr(_i32(o["nn_ba"])), _ptr(_f32(o["d_ba"])),
          _ptr(_f64(o["loss"], "loss")), _ptr(add), _ptr(ws), ws.numel(), _opts(kernel, batch, seed, warm=warm),
          _stream())
    o["means"], o["total"] = o["loss"][0:2], o["loss"][2:3]
    return o


def point_mesh_backward(verts, faces, queries, rec, scale, g_verts=None, g_loss=None):
    """g_verts += scale * g * d(sum_q d^2_q)/dV from closest-point records rec (face, point, bary);
    g = g_loss (a float64 device scalar) or 1."""
    if g_verts is None:
        g_verts = torch.zeros_like(verts)
    _call("mg_point_mesh_backward", _ptr(verts), verts.shape[1], _ptr(faces), faces.shape[1], _ptr(queries),
          queries.shape[1], _ptr(rec["face"]), _ptr(rec["point"]), _ptr(rec["bary"]), float(scale),
          _ptr(_f64(g_loss)), _ptr(g_verts), _stream())
    return g_verts


def chamfer_backward(a, b, nn_ab, nn_ba, scale_ab, scale_ba, g_a=None, g_loss=None):
    """g_a += g * gradient of scale_ab * sum d_ab + scale_ba * sum d_ba w.r.t. a (g = g_loss or 1)."""
    if g_a is None:
        g_a = torch.zeros_like(a)
    _call("mg_chamfer_backward", _ptr(a), a.shape[1], _ptr(b), b.shape[1], _ptr(nn_ab), _ptr(nn_ba),
          float(scale_ab), float(scale_ba), _ptr(_f64(g_loss)), _ptr(g_a), _stream())
    return g_a


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float32 device tensors (step counts from 1)."""
    _call("mg_adam_step", _ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), int(step), float(lr),
          float(beta1), float(beta2), float(eps), _stream())
    return param


def validate_indices(idx, bound, status):
    _call("mg_validate_indices", _ptr(_i32(idx)), idx.numel(), int(bound), _ptr(status), _stream())
    return status


def validate_finite(x, status):
    _call("mg_validate_finite", _ptr(_f32(x)), x.numel(), _ptr(status), _stream())
    return status
