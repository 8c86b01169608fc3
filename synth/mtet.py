"""Varying-topology targets.

* marching_tetrahedra: iso-surface of a sampled scalar field on a regular grid.
  Each grid cube is split into the 6 tetrahedra of the Freudenthal (Kuhn)
  decomposition along its main diagonal, which is conforming across cubes; the
  16-case tetrahedron table is generated below from the sign pattern rather than
  typed in.  Surface vertices sit on grid edges by linear interpolation and are
  shared between all triangles that cut the same edge.  Triangles face +grad(phi).
  No marching-cubes library exists in this environment; marching tetrahedra
  yields roughly 2-3x the triangles of marching cubes at equal grid spacing.
* radial_level_set_target: the zero set of |x| - R(x/|x|, t) of a radial shape,
  i.e. the same continuous surface the fixed-topology frames sample.
* split_faces_target: doubles a mesh's face count by splitting every face at the
  midpoint of one seeded-random edge (no vertex dedup), so connectivity changes
  every frame.
"""

import itertools

import numpy as np

# Freudenthal split: one tetrahedron per permutation of the axes, walking from
# corner (0,0,0) to corner (1,1,1) one axis at a time.
_TETS = []
for perm in itertools.permutations(range(3)):
    c = [0, 0, 0]
    corners = [tuple(c)]
    for ax in perm:
        c[ax] = 1
        corners.append(tuple(c))
    _TETS.append(corners)


def _case_table():
    """For each 4-bit inside mask, the triangles as triples of (inside, outside) tet-vertex pairs."""
    table = {}
    for mask in range(16):
        ins = [i for i in range(4) if mask >> i & 1]
        outs = [i for i in range(4) if not mask >> i & 1]
        if len(ins) in (0, 4):
            table[mask] = []
        elif len(ins) == 1:
            a = ins[0]
            table[mask] = [((a, outs[0]), (a, outs[1]), (a, outs[2]))]
        elif len(ins) == 3:
            d = outs[0]
            table[mask] = [((ins[0], d), (ins[1], d), (ins[2], d))]
        else:
            a, b = ins
            c, d = outs
            # cyclic order around the quad: ac, ad, bd, bc
            table[mask] = [((a, c), (a, d), (b, d)), ((a, c), (b, d), (b, c))]
    return table


_CASES = _case_table()


def marching_tetrahedra(phi, lo, h):
    """Iso-surface phi == 0 of a grid field phi[(n+1),(n+1),(n+1)] with origin lo and spacing h.

    Returns (V, F) AoS float64 / int64.  Field values within 1e-3 h of zero are
    moved to +1e-3 h, so surface vertices stay at least 1e-3 h away from grid
    vertices and no triangle collapses to zero area in float32.
    """
    eps = 1e-3 * h
    phi = np.where(np.abs(phi) < eps, eps, phi)
    n1 = phi.shape[0]
    n = n1 - 1
    flat = phi.reshape(-1)
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = ((ii * n1 + jj) * n1 + kk).reshape(-1)

    def corner_id(c):
        return base + (c[0] * n1 + c[1]) * n1 + c[2]

    edge_a, edge_b, tri_edges = [], [], []
    n_edges = 0
    for corners in _TETS:
        gid = np.stack([corner_id(c) for c in corners])          # [4][cubes]
        inside = flat[gid] < 0.0
        mask = (inside * (1 << np.arange(4))[:, None]).sum(0)
        for m in range(1, 15):
            sel = np.nonzero(mask == m)[0]
            if sel.size == 0:
                continue
            for tri in _CASES[m]:
                ids = []
                for (a, b) in tri:
                    edge_a.append(gid[a, sel])
                    edge_b.append(gid[b, sel])
                    ids.append(np.arange(n_edges, n_edges + sel.size))
                    n_edges += sel.size
                tri_edges.append(np.stack(ids, 1))
    if not tri_edges:
        return np.zeros((0, 3)), np.zeros((0, 3), np.int64)
    ea = np.concatenate(edge_a)      # inside end
    eb = np.concatenate(edge_b)      # outside end
    te = np.concatenate(tri_edges)
    lo_id = np.minimum(ea, eb)
    hi_id = np.maximum(ea, eb)
    key = lo_id * flat.size + hi_id
    ukey, inv = np.unique(key, return_inverse=True)
    ua = ukey // flat.size
    ub = ukey % flat.size

    def pos(g):
        k = g % n1
        j = (g // n1) % n1
        i = g // (n1 * n1)
        return lo + h * np.stack([i, j, k], 1).astype(np.float64)

    fa, fb = flat[ua], flat[ub]
    t = fa / (fa - fb)
    verts = pos(ua) + t[:, None] * (pos(ub) - pos(ua))
    faces = inv[te]
    # orient each triangle so that its normal points from inside to outside
    p0, p1, p2 = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    tri0 = te[:, 0]
    outdir = pos(eb[tri0]) - pos(ea[tri0])
    flip = (nrm * outdir).sum(1) < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    # drop triangles that interpolation made degenerate (coincident vertices)
    keep = (faces[:, 0] != faces[:, 1]) & (faces[:, 1] != faces[:, 2]) & (faces[:, 0] != faces[:, 2])
    return verts, faces[keep].astype(np.int64)


def radial_level_set_target(shape, motion, t, n_cells, extent=1.4):
    """Marching-tetrahedra mesh of the surface |x| = r(x^) + u(x^, t) on an n_cells^3 grid."""
    g = np.linspace(-extent, extent, n_cells + 1)
    h = g[1] - g[0]
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    nr = np.linalg.norm(x, axis=1)
    xhat = x / np.where(nr > 0, nr, 1.0)[:, None]
    xhat[nr == 0] = [0.0, 0.0, 1.0]
    R = shape.radius(xhat)
    if motion is not None:
        R = R + motion.offset(xhat, float(t))
    phi = (nr - R).reshape(n_cells + 1, n_cells + 1, n_cells + 1)
    return marching_tetrahedra(phi, np.array([-extent] * 3), h)


def split_faces_target(v, f, rng):
    """Split each face (a, b, c) at the midpoint m of a random edge into two faces.

    A corner k is drawn per face; the edge opposite k is split, giving faces
    (k, k+1, m) and (k, m, k+2) in the face's cyclic order.  Every face adds its
    own midpoint vertex: |V'| = |V| + |F|, |F'| = 2 |F|.
    """
    nf = f.shape[0]
    k = rng.integers(0, 3, nf)
    r = np.arange(nf)
    a = f[r, k]
    b = f[r, (k + 1) % 3]
    c = f[r, (k + 2) % 3]
    m = v.shape[0] + r
    mid = 0.5 * (v[b] + v[c])
    v2 = np.concatenate([v, mid])
    f2 = np.concatenate([np.stack([a, b, m], 1), np.stack([a, m, c], 1)])
    return v2, f2.astype(np.int64)
