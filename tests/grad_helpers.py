"""Oracle gradients for the GPU gradient tests, evaluated at the device's argmins."""

import numpy as np

from gpu_helpers import scale_of
from oracle import closest as oc
from oracle import losses as olo


def normwise(a, b, scale=None):
    """|a - b| / |b| (2-norms), or / scale when given."""
    b = np.asarray(b, np.float64)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (np.linalg.norm(b) if scale is None else scale)


def oracle_grad_at(V, F, B, Y, argmins, parts=False):
    """Oracle loss and analytic gradient at V, evaluated at the device's argmins
    (face, nn_ab, nn_ba) after checking that each of them ties the oracle's own
    minimum within the position tolerance: a gradient of a min is only defined up
    to the choice among tied minimisers.

    parts=True also returns the sum of the norms of the gradients of the loss's
    three terms (P, CD a->b, CD b->a).  Float32 rounding error scales with those
    terms, not with their sum, which nearly cancels close to an optimum; it is
    the scale of the normwise gradient tolerance there."""
    face, nn_ab, nn_ba = (np.asarray(a).astype(np.int64) for a in argmins)
    L_ref, aux = olo.template_loss(V, F, B, Y)
    Lsc = scale_of(V)
    rec = oc.closest_on_faces(V, F, Y, face)
    tol = 1e-5 * np.maximum(np.sqrt(aux["rec"]["dist2"]), 0.1 * Lsc)
    assert (np.sqrt(rec["dist2"]) <= np.sqrt(aux["rec"]["dist2"]) + tol).all()
    mu = aux["mu"]
    d_ab = ((mu - Y[:, nn_ab]) ** 2).sum(0)
    d_ba = ((mu[:, nn_ba] - Y) ** 2).sum(0)
    _, _, _, r_ab, r_ba = olo.chamfer(mu, Y)
    assert (np.sqrt(d_ab) <= np.sqrt(r_ab) + 1e-5 * np.maximum(np.sqrt(r_ab), 0.1 * Lsc)).all()
    assert (np.sqrt(d_ba) <= np.sqrt(r_ba) + 1e-5 * np.maximum(np.sqrt(r_ba), 0.1 * Lsc)).all()
    g_p = olo.point_to_mesh_grad(V, F, Y, rec)
    g = g_p + olo.binding_vjp(V, F, B, olo.chamfer_grad_a(mu, Y, nn_ab, nn_ba))
    if not parts:
        return L_ref, g
    g_ab = olo.binding_vjp(V, F, B, (2.0 / mu.shape[1]) * (mu - Y[:, nn_ab]))
    g_ba = olo.binding_vjp(V, F, B, olo.chamfer_grad_a(mu, Y, nn_ab, nn_ba)) - g_ab
    scale = np.linalg.norm(g_p) + np.linalg.norm(g_ab) + np.linalg.norm(g_ba)
    return L_ref, g, scale
