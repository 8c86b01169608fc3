"""Closest points on triangles and meshes, float64 brute force.

TEST INFRASTRUCTURE ONLY (see the package docstring).

NearestSurface (Sec. 3.3, Eq. 1 and Eq. 2) projects a point onto a mesh with
barycentric interpolation for sub-face accuracy.  The paper's "k-NN weighted"
variant has no stated k or weights; the reading here is k = 1: the closest
point over all faces, exact ties of the squared distance broken by the lowest
face id.  Outputs: face id, closest point c, barycentrics (w1, w2) of c with
c = (1 - w1 - w2) v0 + w1 v1 + w2 v2, squared distance, and the face's unit
normal computed on demand (Sec. 3.4 step 3).

Closest point on one triangle: Ericson, Real-Time Collision Detection (2005),
Sec. 5.1.5 - classify the point into the Voronoi regions of the vertices,
edges and face from six dot products.  A triangle of zero area (the interior
branch's denominator is not positive) falls back to the nearest of the three
edge segments, ties in the order AB, AC, BC.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmgu_oracle.so")
_lib = None


def build_c(force=False):
    """Compile oracle/cpm.c (plain C, float64) into oracle/libmgu_oracle.so."""
    src = os.path.join(_HERE, "cpm.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               src, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _clib():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_c())
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.oracle_closest_point_mesh.argtypes = [P, I, P, I, P, I, ctypes.c_double, P, P, P, P]
        lib.oracle_closest_point_mesh.restype = ctypes.c_int
        lib.oracle_nearest_points.argtypes = [P, I, P, I, P, P]
        lib.oracle_nearest_points.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def set_threads(n):
    """OpenMP threads of the plain-C brute force (a timing knob; results do not change)."""
    _clib().oracle_set_threads(int(n))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dot(a, b):
    return (a * b).sum(-1)


def _segment(p, a, b):
    ab = b - a
    den = _dot(ab, ab)
    t = np.where(den > 0, _dot(p - a, ab) / np.where(den > 0, den, 1.0), 0.0)
    t = np.clip(t, 0.0, 1.0)
    return a + t[..., None] * ab, t


def closest_on_triangle(p, a, b, c):
    """Closest point on triangles abc to points p (broadcasting [...,3]).

    Returns (point [...,3], weights [...,3]) with point = w0 a + w1 b + w2 c.
    """
    p, a, b, c = np.broadcast_arrays(*(np.asarray(x, dtype=np.float64) for x in (p, a, b, c)))
    shape = p.shape[:-1]
    ab, ac, ap = b - a, c - a, p - a
    bp, cp = p - b, p - c
    d1, d2 = _dot(ab, ap), _dot(ac, ap)
    d3, d4 = _dot(ab, bp), _dot(ac, bp)
    d5, d6 = _dot(ab, cp), _dot(ac, cp)
    vc = d1 * d4 - d3 * d2
    vb = d5 * d2 - d1 * d6
    va = d3 * d6 - d5 * d4

    w = np.zeros(shape + (3,))
    # A triangle of zero area is a segment or a point (the hull of collinear vertices):
    # the region tests below assume a proper triangle, so it takes the edge fallback.
    nrm = np.cross(ab, ac)
    flat = _dot(nrm, nrm) == 0
    done = flat.copy()

    def take(mask, w0, w1, w2):
        nonlocal done
        m = mask & ~done
        w[m, 0], w[m, 1], w[m, 2] = w0[m], w1[m], w2[m]
        done = done | m

    one, zero = np.ones(shape), np.zeros(shape)
    take((d1 <= 0) & (d2 <= 0), one, zero, zero)                         # vertex A
    take((d3 >= 0) & (d4 <= d3), zero, one, zero)                        # vertex B
    m = (vc <= 0) & (d1 >= 0) & (d3 <= 0)                                # edge AB
    v = np.where(m & ~done, d1 / np.where(d1 - d3 != 0, d1 - d3, 1.0), 0.0)
    take(m, 1 - v, v, zero)
    take((d6 >= 0) & (d5 <= d6), zero, zero, one)                        # vertex C
    m = (vb <= 0) & (d2 >= 0) & (d6 <= 0)                                # edge AC
    t = np.where(m & ~done, d2 / np.where(d2 - d6 != 0, d2 - d6, 1.0), 0.0)
    take(m, 1 - t, zero, t)
    e43, e56 = d4 - d3, d5 - d6
    m = (va <= 0) & (e43 >= 0) & (e56 >= 0)                              # edge BC
    t = np.where(m & ~done, e43 / np.where(e43 + e56 != 0, e43 + e56, 1.0), 0.0)
    take(m, zero, 1 - t, t)
    den = va + vb + vc
    interior = ~done & (den > 0)                                         # face interior
    dd = np.where(interior, den, 1.0)
    take(interior, 1 - vb / dd - vc / dd, vb / dd, vc / dd)
    pt = w[..., 0:1] * a + w[..., 1:2] * b + w[..., 2:3] * c
    rest = ~done | flat                                                  # zero-area fallback
    if rest.any():
        best = None
        for (u, s, iu, is_) in ((a, b, 0, 1), (a, c, 0, 2), (b, c, 1, 2)):
            q, tt = _segment(p, u, s)
            dq = _dot(p - q, p - q)
            if best is None:
                best, bq, bw = dq, q, np.zeros(shape + (3,))
                bw[..., iu], bw[..., is_] = 1 - tt, tt
            else:
                better = dq < best
                best = np.where(better, dq, best)
                bq = np.where(better[..., None], q, bq)
                nw = np.zeros(shape + (3,))
                nw[..., iu], nw[..., is_] = 1 - tt, tt
                bw = np.where(better[..., None], nw, bw)
        pt[rest], w[rest] = bq[rest], bw[rest]
    return pt, w


def _tri_normals(a, b, c):
    n = np.cross(b - a, c - a)
    e1 = np.linalg.norm(b - a, axis=-1)
    ln = np.linalg.norm(n, axis=-1)
    ok = (ln > 0) & (e1 > 0)
    return np.where(ok[..., None], n / np.where(ok, ln, 1.0)[..., None], 0.0)


def closest_point_mesh(verts, faces, queries, max_dist2=np.inf, chunk=None, impl="c"):
    """Brute force over all faces for every query.

    verts [3][V], faces [3][F], queries [3][Q].  Returns dict: face [Q] int64
    (-1 if nothing within max_dist2), point [3][Q], bary [2][Q] (w1, w2),
    dist2 [Q] (+inf if none), normal [3][Q] (zero if none).  impl "c" runs the
    plain-C loop in cpm.c, impl "numpy" the vectorised version below; the two are
    independent codings of the same definition.
    """
    if impl == "c":
        return _closest_point_mesh_c(verts, faces, queries, max_dist2)
    V = np.asarray(verts, dtype=np.float64).T
    F = np.asarray(faces).astype(np.int64).T
    Q = np.asarray(queries, dtype=np.float64).T
    nq, nf = Q.shape[0], F.shape[0]
    face = np.full(nq, -1, np.int64)
    point = Q.copy()
    bary = np.zeros((nq, 2))
    d2 = np.full(nq, np.inf)
    normal = np.zeros((nq, 3))
    if nq == 0 or nf == 0:
        return {"face": face, "point": point.T, "bary": bary.T, "dist2": d2, "normal": normal.T}
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    if chunk is None:
        chunk = max(1, int(2_000_000 // max(nf, 1)))
    for s in range(0, nq, chunk):
        p = Q[s:s + chunk, None, :]
        pt, w = closest_on_triangle(p, a[None], b[None], c[None])
        dd = _dot(p - pt, p - pt)                     # [chunk, F]
        k = np.argmin(dd, axis=1)                     # first minimum = lowest face id
        r = np.arange(k.size)
        best = dd[r, k]
        ok = best <= max_dist2
        idx = np.arange(s, s + k.size)[ok]
        kk = k[ok]
        face[idx] = kk
        point[idx] = pt[r[ok], kk]
        bary[idx] = w[r[ok], kk][:, 1:]
        d2[idx] = best[ok]
        normal[idx] = _tri_normals(a[kk], b[kk], c[kk])
    return {"face": face, "point": point.T, "bary": bary.T, "dist2": d2, "normal": normal.T}


def _closest_point_mesh_c(verts, faces, queries, max_dist2):
    V = np.ascontiguousarray(verts, dtype=np.float64)
    F = np.ascontiguousarray(faces, dtype=np.int64)
    Q = np.ascontiguousarray(queries, dtype=np.float64)
    nq, nf = Q.shape[1], F.shape[1]
    face = np.empty(nq, np.int64)
    point = np.empty((3, nq))
    bary = np.empty((2, nq))
    d2 = np.empty(nq)
    rc = _clib().oracle_closest_point_mesh(_ptr(V), V.shape[1], _ptr(F), nf, _ptr(Q), nq,
                                           float(max_dist2), _ptr(face), _ptr(point), _ptr(bary), _ptr(d2))
    if rc != 0:
        raise ValueError("face index out of range")
    normal = np.zeros((3, nq))
    hit = face >= 0
    if hit.any():
        tri = F[:, face[hit]]
        a, b, c = V[:, tri[0]].T, V[:, tri[1]].T, V[:, tri[2]].T
        normal[:, hit] = _tri_normals(a, b, c).T
    return {"face": face, "point": point, "bary": bary, "dist2": d2, "normal": normal}


def closest_on_faces(verts, faces, queries, face_ids):
    """Closest-point records of each query on one given face each (float64).

    Used to evaluate the oracle at another implementation's argmins once those
    are shown to be ties of the oracle's own minimum.
    """
    V = np.asarray(verts, dtype=np.float64).T
    fid = np.asarray(face_ids, dtype=np.int64)
    F = np.asarray(faces).astype(np.int64).T[fid]
    p = np.asarray(queries, dtype=np.float64).T
    pt, w = closest_on_triangle(p, V[F[:, 0]], V[F[:, 1]], V[F[:, 2]])
    return {"face": fid, "point": pt.T.copy(), "bary": w[:, 1:].T.copy(), "dist2": _dot(p - pt, p - pt),
            "normal": _tri_normals(V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]).T.copy()}


def distances_to_faces(verts, faces, queries, face_ids):
    """Squared distance from each query to one given face each (for tie checks)."""
    V = np.asarray(verts, dtype=np.float64).T
    F = np.asarray(faces).astype(np.int64).T[np.asarray(face_ids, dtype=np.int64)]
    p = np.asarray(queries, dtype=np.float64).T
    pt, _ = closest_on_triangle(p, V[F[:, 0]], V[F[:, 1]], V[F[:, 2]])
    return _dot(p - pt, p - pt)


def nearest_points(src, dst, chunk=None, impl="c"):
    """Brute-force nearest neighbour in dst [3][M] of each src [3][N]: (index [N], dist2 [N]).

    Exact ties go to the lowest index.
    """
    if impl == "c":
        A = np.ascontiguousarray(src, dtype=np.float64)
        B = np.ascontiguousarray(dst, dtype=np.float64)
        idx = np.empty(A.shape[1], np.int64)
        d2 = np.empty(A.shape[1])
        if A.shape[1] and B.shape[1]:
            _clib().oracle_nearest_points(_ptr(A), A.shape[1], _ptr(B), B.shape[1], _ptr(idx), _ptr(d2))
        else:
            idx[:] = -1
            d2[:] = np.inf
        return idx, d2
    A = np.asarray(src, dtype=np.float64).T
    B = np.asarray(dst, dtype=np.float64).T
    n, m = A.shape[0], B.shape[0]
    idx = np.full(n, -1, np.int64)
    d2 = np.full(n, np.inf)
    if n == 0 or m == 0:
        return idx, d2
    if chunk is None:
        chunk = max(1, int(4_000_000 // m))
    for s in range(0, n, chunk):
        p = A[s:s + chunk, None, :]
        dd = ((p - B[None]) ** 2).sum(-1)
        k = np.argmin(dd, axis=1)
        idx[s:s + k.size] = k
        d2[s:s + k.size] = dd[np.arange(k.size), k]
    return idx, d2


def template_projection(template_verts, target_verts, target_faces):
    """Eq. 2: every template vertex replaced by its closest point on the target mesh."""
    r = closest_point_mesh(target_verts, target_faces, template_verts)
    return r["point"], r
