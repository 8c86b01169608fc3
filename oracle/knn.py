"""k-NN weighted surface projection (NearestSurface, Sec. 3.3 Eq. 1), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper projects a point onto a mesh "via k-NN weighted surface projection"
without stating k or the weights.  Reading: the k faces nearest to the point
(point-to-triangle distance, ties of the squared distance to the lowest face
id), each with its closest point c_i at distance d_i, combined as
sum w_i c_i / sum w_i with inverse-distance weights w_i = 1 / (d_i + eps).
k = 1 is the single closest point.  Parity with the paper is unpinned (k and
the weights are ours); a face at distance exactly 0 gives its own point.  The
definition itself is pinned by the tests.
"""

import numpy as np

from .closest import closest_on_triangle, closest_on_faces


def knn_faces(verts, faces, queries, k, chunk=2048):
    """The k nearest faces of every query: (face [k][Q] int64, dist2 [k][Q]), sorted
    by (dist2, face id); brute force over all faces."""
    V = np.asarray(verts, dtype=np.float64).T
    F = np.asarray(faces).astype(np.int64).T
    P = np.asarray(queries, dtype=np.float64).T
    nq, nf = P.shape[0], F.shape[0]
    k = int(min(k, nf))
    best_d = np.full((nq, 0), np.inf)
    best_f = np.zeros((nq, 0), np.int64)
    for s in range(0, nf, chunk):
        ids = np.arange(s, min(nf, s + chunk))
        tri = F[ids]
        pt, _ = closest_on_triangle(P[:, None, :], V[tri[:, 0]][None], V[tri[:, 1]][None], V[tri[:, 2]][None])
        d2 = ((P[:, None, :] - pt) ** 2).sum(-1)                      # [Q][chunk]
        cand_d = np.concatenate([best_d, d2], axis=1)
        cand_f = np.concatenate([best_f, np.broadcast_to(ids, d2.shape)], axis=1)
        order = np.lexsort((cand_f, cand_d), axis=1)[:, :k]           # by distance, then face id
        best_d = np.take_along_axis(cand_d, order, axis=1)
        best_f = np.take_along_axis(cand_f, order, axis=1)
    return best_f.T.copy(), best_d.T.copy()


def weighted_point(verts, faces, queries, face_k, eps):
    """sum w_i c_i / sum w_i over the given faces face_k [k][Q] (w_i = 1 / (d_i + eps))."""
    face_k = np.asarray(face_k, dtype=np.int64)
    num = np.zeros((3, face_k.shape[1]))
    den = np.zeros(face_k.shape[1])
    hit = np.zeros(face_k.shape[1], bool)
    on = np.zeros((3, face_k.shape[1]))
    for j in range(face_k.shape[0]):
        r = closest_on_faces(verts, faces, queries, face_k[j])
        first = (r["dist2"] == 0) & ~hit
        on[:, first] = r["point"][:, first]
        hit |= first
        with np.errstate(divide="ignore"):
            w = 1.0 / (np.sqrt(r["dist2"]) + eps)
        num += np.where(np.isfinite(w), w, 0.0) * r["point"]
        den += np.where(np.isfinite(w), w, 0.0)
    out = num / np.where(den > 0, den, 1.0)
    out[:, hit] = on[:, hit]
    return out


def knn_surface(verts, faces, queries, k=4, eps=0.0):
    """k-NN weighted projection of queries [3][Q]: dict face [k][Q], dist2 [k][Q], point [3][Q]."""
    face_k, d2 = knn_faces(verts, faces, queries, k)
    return {"face": face_k, "dist2": d2, "point": weighted_point(verts, faces, queries, face_k, eps)}
