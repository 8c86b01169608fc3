"""Face-bound Gaussians re-posed from their triangles, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper keeps a fixed-topology physics mesh and a Gaussian render
representation in sync (Sec. 3.2) and recomputes per-face normals on demand
(Sec. 3.4 step 3), but never writes down how a Gaussian follows its face.  The
reading used here (binding in the spirit of mesh-anchored Gaussians):

* triangle frame of face (i0, i1, i2) in stored order: e1 = v1 - v0,
  e2 = v2 - v0, n = e1 x e2, t = e1 / |e1|, nh = n / |n|, b = nh x t,
  R_f = [t b nh] (columns).  Degenerate (|e1| == 0 or |n| == 0 exactly):
  R_f = I and the normal is the zero vector.
* mean   mu = b0 v0 + b1 v1 + b2 v2 + delta nh with b0 = 1 - b1 - b2.
* rotation  R_g = R_f R(q_l), q_l a Hamilton quaternion (w, x, y, z), normalised;
  the output quaternion is Shepperd's (1978) extraction from R_g with the sign
  fixed so that w > 0 (or, when w == 0, the first non-zero of x, y, z is > 0).
* covariance  Sigma = R_g diag(s^2) R_g^T with s = exp(log_scale), packed as
  (xx, xy, xz, yy, yz, zz).
Parity of this formula with the paper is unpinned (the paper has none); it is
pinned by invariants (rigid-motion equivariance, eigenvalues, rest pose).
"""

import numpy as np


def _aos(x):
    return np.asarray(x, dtype=np.float64).T


def triangle_frame(v0, v1, v2):
    """R_f [N,3,3] (columns t, b, nh), unit normal nh [N,3], degenerate flag [N]."""
    e1 = v1 - v0
    e2 = v2 - v0
    n = np.cross(e1, e2)
    l1 = np.linalg.norm(e1, axis=1)
    ln = np.linalg.norm(n, axis=1)
    deg = (l1 == 0.0) | (ln == 0.0)
    l1s = np.where(deg, 1.0, l1)
    lns = np.where(deg, 1.0, ln)
    t = e1 / l1s[:, None]
    nh = n / lns[:, None]
    b = np.cross(nh, t)
    R = np.stack([t, b, nh], axis=2)
    R[deg] = np.eye(3)
    nh[deg] = 0.0
    return R, nh, deg


def quat_to_matrix(q):
    """Rotation matrices [N,3,3] of Hamilton quaternions q [N,4] = (w, x, y, z) (unit)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def canonical_sign(q):
    """Flip q [N,4] so that w > 0, or if w == 0 the first non-zero of (x, y, z) is positive."""
    q = q.copy()
    lead = q[:, 0].copy()
    for k in (1, 2, 3):
        lead = np.where(lead == 0.0, q[:, k], lead)
    q[lead < 0] *= -1.0
    return q


def matrix_to_quat(R):
    """Shepperd (1978): unit quaternion (w, x, y, z) of rotation matrices R [N,3,3].

    The largest of (trace, R00, R11, R22) picks which component is taken from a
    square root; the other three follow from sums/differences of off-diagonals.
    """
    r00, r11, r22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    tr = r00 + r11 + r22
    pick = np.argmax(np.stack([tr, r00, r11, r22], 1), axis=1)
    q = np.empty((R.shape[0], 4))
    m = pick == 0
    if m.any():
        w = 0.5 * np.sqrt(1.0 + tr[m])
        f = 0.25 / w
        q[m] = np.stack([w, (R[m, 2, 1] - R[m, 1, 2]) * f, (R[m, 0, 2] - R[m, 2, 0]) * f,
                         (R[m, 1, 0] - R[m, 0, 1]) * f], 1)
    m = pick == 1
    if m.any():
        x = 0.5 * np.sqrt(1.0 + r00[m] - r11[m] - r22[m])
        f = 0.25 / x
        q[m] = np.stack([(R[m, 2, 1] - R[m, 1, 2]) * f, x, (R[m, 0, 1] + R[m, 1, 0]) * f,
                         (R[m, 0, 2] + R[m, 2, 0]) * f], 1)
    m = pick == 2
    if m.any():
        y = 0.5 * np.sqrt(1.0 - r00[m] + r11[m] - r22[m])
        f = 0.25 / y
        q[m] = np.stack([(R[m, 0, 2] - R[m, 2, 0]) * f, (R[m, 0, 1] + R[m, 1, 0]) * f, y,
                         (R[m, 1, 2] + R[m, 2, 1]) * f], 1)
    m = pick == 3
    if m.any():
        z = 0.5 * np.sqrt(1.0 - r00[m] - r11[m] + r22[m])
        f = 0.25 / z
        q[m] = np.stack([(R[m, 1, 0] - R[m, 0, 1]) * f, (R[m, 0, 2] + R[m, 2, 0]) * f,
                         (R[m, 1, 2] + R[m, 2, 1]) * f, z], 1)
    return canonical_sign(q)


def pack_sym(S):
    """(xx, xy, xz, yy, yz, zz) [6][N] of symmetric matrices S [N,3,3]."""
    return np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]])


def unpack_sym(p):
    """Symmetric matrices [N,3,3] from packed (xx, xy, xz, yy, yz, zz) [6][N]."""
    p = np.asarray(p, dtype=np.float64)
    S = np.empty((p.shape[1], 3, 3))
    S[:, 0, 0], S[:, 1, 1], S[:, 2, 2] = p[0], p[3], p[5]
    S[:, 0, 1] = S[:, 1, 0] = p[1]
    S[:, 0, 2] = S[:, 2, 0] = p[2]
    S[:, 1, 2] = S[:, 2, 1] = p[4]
    return S


def repose(verts, faces, binding, offset=None):
    """Re-pose every Gaussian on its face.

    verts [3][V], faces [3][F], binding with face [G], bary [2][G] = (b1, b2),
    q_local [4][G] = (w, x, y, z), log_scale [3][G]; offset [G] (normal offset
    delta) or None for zero.  Returns dict of float64 arrays: mean [3][G],
    rot [G,3,3] (R_g), quat [4][G], cov [6][G], normal [3][G] (face unit normal),
    degenerate [G].
    """
    V = _aos(verts)
    F = np.asarray(faces).T.astype(np.int64)
    fid = np.asarray(binding["face"]).astype(np.int64)
    tri = F[fid]
    v0, v1, v2 = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    Rf, nh, deg = triangle_frame(v0, v1, v2)
    b = np.asarray(binding["bary"], dtype=np.float64)
    b1, b2 = b[0], b[1]
    b0 = 1.0 - b1 - b2
    mu = b0[:, None] * v0 + b1[:, None] * v1 + b2[:, None] * v2
    if offset is not None:
        mu = mu + np.asarray(offset, dtype=np.float64)[:, None] * nh
    ql = np.asarray(binding["q_local"], dtype=np.float64).T
    ql = ql / np.linalg.norm(ql, axis=1, keepdims=True)
    Rg = Rf @ quat_to_matrix(ql)
    s2 = np.exp(2.0 * np.asarray(binding["log_scale"], dtype=np.float64)).T     # [G,3]
    cov = (Rg * s2[:, None, :]) @ np.transpose(Rg, (0, 2, 1))
    return {
        "mean": mu.T.copy(),
        "rot": Rg,
        "quat": matrix_to_quat(Rg).T.copy(),
        "cov": pack_sym(cov),
        "normal": nh.T.copy(),
        "degenerate": deg,
    }


def bind_rest_pose(verts0, faces, face, mean0, quat0, log_scale):
    """Inverse of repose on the rest mesh: world-space Gaussians -> binding.

    mean0 [3][G] is projected onto its face's plane: its barycentrics in that
    plane give (b1, b2) and its signed distance along nh gives delta;
    q_l = quat(R_f^T R(q0)).  Returns (binding dict, offset [G]), float64.
    """
    V = _aos(verts0)
    F = np.asarray(faces).T.astype(np.int64)
    fid = np.asarray(face).astype(np.int64)
    tri = F[fid]
    v0, v1, v2 = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    Rf, nh, _ = triangle_frame(v0, v1, v2)
    m = _aos(mean0)
    delta = ((m - v0) * nh).sum(1)
    p = m - delta[:, None] * nh
    e1, e2, d = v1 - v0, v2 - v0, p - v0
    g11, g12, g22 = (e1 * e1).sum(1), (e1 * e2).sum(1), (e2 * e2).sum(1)
    r1, r2 = (d * e1).sum(1), (d * e2).sum(1)
    det = g11 * g22 - g12 * g12
    b1 = (g22 * r1 - g12 * r2) / det
    b2 = (g11 * r2 - g12 * r1) / det
    q0 = _aos(quat0)
    q0 = q0 / np.linalg.norm(q0, axis=1, keepdims=True)
    Rl = np.transpose(Rf, (0, 2, 1)) @ quat_to_matrix(q0)
    binding = {
        "face": fid,
        "bary": np.stack([b1, b2]),
        "q_local": matrix_to_quat(Rl).T.copy(),
        "log_scale": np.asarray(log_scale, dtype=np.float64),
    }
    return binding, delta
