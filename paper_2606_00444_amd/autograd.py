"""Differentiable template projection: torch.autograd.Function wrappers.

The paper projects a fixed-topology template onto each reconstructed mesh by
closest points (Sec. 3.3, Eq. 2).  The library also makes that projection a
loss that can be minimised over the template vertices V:

    L(V) = P(V) + CD(mu(V), Y)
    P(V)      = mean over targets y of the squared distance from y to the mesh (V, F)
    CD(A, B)  = mean_a min_b |a - b|^2 + mean_b min_a |a - b|^2
    mu(V)     = the means of the face-bound Gaussians re-posed on (V, F)

Each Function runs its forward and its hand-written backward in libmgu.so
kernels; the upstream gradient of a scalar loss is read on the device (no host
synchronisation).  Minimum-distance terms are differentiated with the argmin
held fixed (Danskin), which is the gradient wherever the argmin is unique.
Float32 atomics accumulate the scatters, so gradients are reproducible to
rounding, not bitwise.  Targets are constants for P; Chamfer differentiates
both point sets.
"""

import torch

from . import api


def _zeros(like):
    return api.fill(torch.empty_like(like), 0.0)


class MeshGaussianBinding(torch.autograd.Function):
    """(mean [3][G], rot [9][G], cov [6][G]) of the face-bound Gaussians on (verts, faces).

    apply(verts, faces, gface, bary, q_local, log_scale, offset=None, frame=True);
    with frame=False only the mean is computed and returned.  Differentiable
    w.r.t. verts (the binding parameters are constants here).
    """

    @staticmethod
    def forward(ctx, verts, faces, gface, bary, q_local, log_scale, offset=None, frame=True):
        ctx.set_materialize_grads(False)
        v = verts.detach()
        o = api.mesh_gaussian_update(v, faces, gface, bary, q_local, log_scale, offset, quat=False, cov=frame,
                                     rot=frame)
        ctx.save_for_backward(v, faces, gface, bary, q_local, log_scale, offset)
        ctx.frame = frame
        return (o["mean"], o["rot"], o["cov"]) if frame else o["mean"]

    @staticmethod
    def backward(ctx, *grads):
        if not ctx.needs_input_grad[0]:
            return (None,) * 8
        v, faces, gface, bary, q_local, log_scale, offset = ctx.saved_tensors
        g_mean = grads[0]
        g_rot = grads[1] if ctx.frame else None
        g_cov = grads[2] if ctx.frame else None
        gv = _zeros(v)
        c = lambda t: None if t is None else t.contiguous()
        api.mesh_gaussian_update_backward(v, faces, gface, bary, q_local, log_scale, offset, c(g_mean), c(g_rot),
                                          c(g_cov), g_verts=gv)
        return (gv,) + (None,) * 7


class PointToMeshLoss(torch.autograd.Function):
    """P(V): mean squared distance from targets [3][Y] to the mesh (verts, faces), a float64 scalar.

    apply(verts, faces, targets, bvh, query=None): bvh is a triangle LBVH over
    faces (built once from any pose of the same topology); it is refit in place
    to verts.  query: traversal options for closest_point_query.
    """

    @staticmethod
    def forward(ctx, verts, faces, targets, bvh, query=None):
        if targets.requires_grad:
            raise ValueError("PointToMeshLoss treats targets as constants")
        v = verts.detach()
        api.lbvh_refit(bvh, v)
        rec = api.closest_point_query(bvh, v, targets, **(query or {}))
        loss = api.mean(rec["dist2"]).reshape(())
        ctx.save_for_backward(v, faces, targets, rec["face"], rec["point"], rec["bary"])
        return loss

    @staticmethod
    def backward(ctx, g):
        if not ctx.needs_input_grad[0]:
            return (None,) * 5
        v, faces, targets, face, point, bary = ctx.saved_tensors
        gv = _zeros(v)
        nq = targets.shape[1]
        if nq:
            api.point_mesh_backward(v, faces, targets, {"face": face, "point": point, "bary": bary}, 1.0 / nq,
                                    gv, g_loss=g.detach().to(torch.float64).contiguous())
        return gv, None, None, None, None


class ChamferLoss(torch.autograd.Function):
    """CD(a, b) (float64 scalar) for point sets a [3][A], b [3][B].

    apply(a, b, bvh_b=None, query=None): a point LBVH over a is built per call;
    bvh_b, if given, is a point LBVH over b (build it once when b is fixed).
    """

    @staticmethod
    def forward(ctx, a, b, bvh_b=None, query=None):
        a_, b_ = a.detach(), b.detach()
        bvh_a = api.lbvh_build(a_, None)
        if bvh_b is None:
            bvh_b = api.lbvh_build(b_, None)
        o = api.chamfer(a_, bvh_a, b_, bvh_b, **(query or {}))
        ctx.save_for_backward(a_, b_, o["nn_ab"], o["nn_ba"])
        return o["total"].reshape(())

    @staticmethod
    def backward(ctx, g):
        a, b, nn_ab, nn_ba = ctx.saved_tensors
        na, nb = a.shape[1], b.shape[1]
        gl = g.detach().to(torch.float64).contiguous()
        ga = gb = None
        if ctx.needs_input_grad[0] and na:
            ga = api.chamfer_backward(a, b, nn_ab, nn_ba, 1.0 / na, 1.0 / nb if nb else 0.0, _zeros(a), g_loss=gl)
        if ctx.needs_input_grad[1] and nb:
            gb = api.chamfer_backward(b, a, nn_ba, nn_ab, 1.0 / nb, 1.0 / na if na else 0.0, _zeros(b), g_loss=gl)
        return ga, gb, None, None


class TemplateProjectionLoss(torch.autograd.Function):
    """L(V) = P(V) + CD(mu(V), Y) (float64 scalar) in one Function: the point-to-mesh
    term, the Gaussian means, the Chamfer term and their sum (mg_chamfer's total with P
    folded in) all come from library calls, and so does the backward.

    apply(verts, faces, gface, bary, q_local, log_scale, offset, targets, bvh,
    targets_bvh=None, query=None, nn_query=None)."""

    @staticmethod
    def forward(ctx, verts, faces, gface, bary, q_local, log_scale, offset, targets, bvh, targets_bvh=None,
                query=None, nn_query=None):
        if targets.requires_grad:
            raise ValueError("TemplateProjectionLoss treats targets as constants")
        v = verts.detach()
        api.lbvh_refit(bvh, v)
        rec = api.closest_point_query(bvh, v, targets, **(query or {}))
        P = api.mean(rec["dist2"])
        mu = api.mesh_gaussian_update(v, faces, gface, bary, q_local, log_scale, offset, quat=False,
                                      cov=False)["mean"]
        bvh_mu = api.lbvh_build(mu, None)
        bvh_y = targets_bvh if targets_bvh is not None else api.lbvh_build(targets, None)
        o = api.chamfer(mu, bvh_mu, targets, bvh_y, add=P, **(nn_query or {}))
        ctx.save_for_backward(v, faces, gface, bary, q_local, log_scale, offset, targets, rec["face"],
                              rec["point"], rec["bary"], mu, o["nn_ab"], o["nn_ba"])
        return o["total"].reshape(())

    @staticmethod
    def backward(ctx, g):
        if not ctx.needs_input_grad[0]:
            return (None,) * 12
        v, faces, gface, bary, q_local, log_scale, offset, targets, face, point, bq, mu, nn_ab, nn_ba = \
            ctx.saved_tensors
        gl = g.detach().to(torch.float64).contiguous()
        gv = _zeros(v)
        ny, G = targets.shape[1], mu.shape[1]
        if ny:
            api.point_mesh_backward(v, faces, targets, {"face": face, "point": point, "bary": bq}, 1.0 / ny, gv,
                                    g_loss=gl)
        if G:
            gmu = api.chamfer_backward(mu, targets, nn_ab, nn_ba, 1.0 / G, 1.0 / ny if ny else 0.0, _zeros(mu),
                                       g_loss=gl)
            api.mesh_gaussian_update_backward(v, faces, gface, bary, q_local, log_scale, offset, gmu, g_verts=gv)
        return (gv,) + (None,) * 11


def template_projection_loss(verts, faces, binding, targets, bvh, targets_bvh=None, query=None, nn_query=None):
    """L(V) = P(V) + CD(mu(V), Y) as a differentiable float64 scalar.

    binding: dict with face, bary, q_local, log_scale (and optionally offset)
    device tensors; bvh: triangle LBVH over faces (refit in place);
    targets_bvh: optional point LBVH over targets.
    """
    return TemplateProjectionLoss.apply(verts, faces, binding["face"], binding["bary"], binding["q_local"],
                                        binding["log_scale"], binding.get("offset"), targets, bvh, targets_bvh,
                                        query, nn_query)
