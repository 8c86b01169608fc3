"""Template-projection losses and their gradients w.r.t. the template vertices, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* P(V)  = mean over targets y of d^2(y, M(V)), M(V) the template mesh
          (template projection, Sec. 3.3 Eq. 2, made a loss).
* CD(A, B) = mean_a min_b |a - b|^2 + mean_b min_a |a - b|^2.  The paper reports
          Chamfer distance (Sec. 4.2) without a formula; reading: squared
          distances, means, both directions, no factor 1/2.
* L(V)  = P(V) + CD(mu(V), Y) with mu(V) the re-posed Gaussian means.

Gradients (Danskin: at a unique argmin the min may be differentiated with the
argmin held fixed):
* dd^2(y)/dv_k = -2 w_k (y - c) for the three vertices of the closest face,
  w the barycentrics of the closest point c;
* dCD/dmu_i = (2/|A|)(mu_i - y_nn(i)) + (2/|B|) sum_{j: nn(j) = i} (mu_i - y_j);
* through the binding, the chain rule over mu = sum_k b_k v_k + delta nh,
  R_g = R_f R_l and Sigma = R_g diag(s^2) R_g^T (see binding_vjp).
"""

import numpy as np

from .closest import closest_point_mesh, nearest_points
from .gaussians import repose, triangle_frame, quat_to_matrix


def point_to_mesh(verts, faces, targets):
    """P(V) and the per-target closest-point records."""
    r = closest_point_mesh(verts, faces, targets)
    return r["dist2"].mean() if r["dist2"].size else 0.0, r


def point_to_mesh_grad(verts, faces, targets, rec=None, scale=None):
    """dP/dV [3][V] (P a mean over targets; scale overrides 1/|Y|)."""
    V = np.asarray(verts, dtype=np.float64)
    F = np.asarray(faces).astype(np.int64)
    Y = np.asarray(targets, dtype=np.float64)
    if rec is None:
        _, rec = point_to_mesh(verts, faces, targets)
    ny = Y.shape[1]
    s = (1.0 / ny) if scale is None else scale
    g = np.zeros_like(V)
    fid = rec["face"]
    w1, w2 = rec["bary"]
    w = np.stack([1 - w1 - w2, w1, w2])
    r = Y - rec["point"]                              # y - c
    for k in range(3):
        for ax in range(3):
            np.add.at(g[ax], F[k, fid], -2.0 * s * w[k] * r[ax])
    return g


def chamfer(a, b):
    """CD(A, B) and the two nearest-neighbour maps (nn_ab: A -> B, nn_ba: B -> A)."""
    nn_ab, d_ab = nearest_points(a, b)
    nn_ba, d_ba = nearest_points(b, a)
    return d_ab.mean() + d_ba.mean(), nn_ab, nn_ba, d_ab, d_ba


def chamfer_grad_a(a, b, nn_ab, nn_ba):
    """dCD/dA [3][|A|] with B held fixed."""
    A = np.asarray(a, dtype=np.float64)
    B = np.asarray(b, dtype=np.float64)
    na, nb = A.shape[1], B.shape[1]
    g = (2.0 / na) * (A - B[:, nn_ab])
    for ax in range(3):
        np.add.at(g[ax], nn_ba, (2.0 / nb) * (A[ax, nn_ba] - B[ax]))
    return g


def binding_vjp(verts, faces, binding, g_mean, g_rot=None, g_cov=None, offset=None):
    """Vector-Jacobian product of repose w.r.t. the vertices: dL/dV [3][V].

    g_mean [3][G] = dL/dmu, g_rot [G,3,3] = dL/dR_g, g_cov [6][G] = dL/d(packed
    Sigma); None means zero.  The quaternion output is not differentiated.
    """
    V = np.asarray(verts, dtype=np.float64).T
    F = np.asarray(faces).astype(np.int64).T
    fid = np.asarray(binding["face"]).astype(np.int64)
    tri = F[fid]
    v0, v1, v2 = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    G = fid.size
    Rf, nh, deg = triangle_frame(v0, v1, v2)
    bb = np.asarray(binding["bary"], dtype=np.float64)
    b = np.stack([1.0 - bb[0] - bb[1], bb[0], bb[1]])
    gm = np.asarray(g_mean, dtype=np.float64).T
    gv = [b[k][:, None] * gm for k in range(3)]

    ql = np.asarray(binding["q_local"], dtype=np.float64).T
    ql = ql / np.linalg.norm(ql, axis=1, keepdims=True)
    Rl = quat_to_matrix(ql)
    Rg = Rf @ Rl
    gR = np.zeros((G, 3, 3)) if g_rot is None else np.asarray(g_rot, dtype=np.float64).copy()
    if g_cov is not None:
        gc = np.asarray(g_cov, dtype=np.float64)
        S = np.empty((G, 3, 3))
        S[:, 0, 0], S[:, 1, 1], S[:, 2, 2] = gc[0], gc[3], gc[5]
        S[:, 0, 1] = S[:, 1, 0] = 0.5 * gc[1]
        S[:, 0, 2] = S[:, 2, 0] = 0.5 * gc[2]
        S[:, 1, 2] = S[:, 2, 1] = 0.5 * gc[4]
        s2 = np.exp(2.0 * np.asarray(binding["log_scale"], dtype=np.float64)).T
        gR = gR + 2.0 * (S @ Rg) * s2[:, None, :]           # (G + G^T) R_g D
    gRf = gR @ np.transpose(Rl, (0, 2, 1))
    g_t, g_b, g_n = gRf[:, :, 0], gRf[:, :, 1], gRf[:, :, 2]
    if offset is not None:
        g_n = g_n + np.asarray(offset, dtype=np.float64)[:, None] * gm
    e1 = v1 - v0
    e2 = v2 - v0
    t = Rf[:, :, 0]
    n = np.cross(e1, e2)
    # b = nh x t
    g_n = g_n + np.cross(t, g_b)
    g_t = g_t + np.cross(g_b, nh)
    l1 = np.linalg.norm(e1, axis=1)
    ln = np.linalg.norm(n, axis=1)
    ok = ~deg
    l1s = np.where(ok, l1, 1.0)
    lns = np.where(ok, ln, 1.0)
    # t = e1/|e1|, nh = n/|n|
    g_e1 = (g_t - (g_t * t).sum(1, keepdims=True) * t) / l1s[:, None]
    g_nn = (g_n - (g_n * nh).sum(1, keepdims=True) * nh) / lns[:, None]
    # n = e1 x e2
    g_e1 = g_e1 + np.cross(e2, g_nn)
    g_e2 = np.cross(g_nn, e1)
    g_e1[~ok] = 0.0
    g_e2[~ok] = 0.0
    gv[1] = gv[1] + g_e1
    gv[2] = gv[2] + g_e2
    gv[0] = gv[0] - g_e1 - g_e2
    out = np.zeros((V.shape[0], 3))
    for k in range(3):
        np.add.at(out, tri[:, k], gv[k])
    return out.T.copy()


def template_loss(verts, faces, binding, targets):
    """L(V) = P(V) + CD(mu(V), Y) and its pieces."""
    P, rec = point_to_mesh(verts, faces, targets)
    mu = repose(verts, faces, binding)["mean"]
    cd, nn_ab, nn_ba, d_ab, d_ba = chamfer(mu, targets)
    return P + cd, {"P": P, "CD": cd, "rec": rec, "mu": mu, "nn_ab": nn_ab, "nn_ba": nn_ba}


def template_loss_grad(verts, faces, binding, targets):
    """dL/dV [3][V] of template_loss (analytic)."""
    L, aux = template_loss(verts, faces, binding, targets)
    g = point_to_mesh_grad(verts, faces, targets, aux["rec"])
    g_mu = chamfer_grad_a(aux["mu"], targets, aux["nn_ab"], aux["nn_ba"])
    g = g + binding_vjp(verts, faces, binding, g_mu)
    return L, g, aux


def central_difference(fun, verts, coords, h):
    """Central differences of scalar fun(verts) at the given (axis, vertex) coordinates."""
    V = np.asarray(verts, dtype=np.float64)
    out = np.empty(len(coords))
    for i, (ax, vi) in enumerate(coords):
        vp = V.copy()
        vm = V.copy()
        vp[ax, vi] += h
        vm[ax, vi] -= h
        out[i] = (fun(vp) - fun(vm)) / (2.0 * h)
    return out
