"""Binary radix tree over sorted Morton codes (Karras 2012) and its bounding boxes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Node numbering follows Karras: internal nodes 0..n-2 (0 is the root), leaves
0..n-1 in sorted order; a child reference c >= 0 is internal node c, c < 0 is
leaf ~c.  Keys are the pairs (code, leaf index), so equal codes still give a
unique tree: delta(i, j) = clz32(k_i xor k_j) if the codes differ, else
32 + clz32(i xor j), and -1 when j is outside [0, n-1].

Bounds (refit): a leaf box is the componentwise min/max of its triangle's three
vertices (or the point itself); an internal box is the union of its children's
boxes.  Refit recomputes every box on the fixed tree and never restructures it
(the paper reuses template-built structures across all frames, Sec. 3.4).
"""

import numpy as np


def clz32(x):
    """Leading zeros of 32-bit unsigned integers (x > 0), by an exact bit-length loop."""
    x = np.asarray(x, dtype=np.uint64)
    bl = np.zeros(x.shape, np.int64)
    for k in range(32):
        bl = np.where((x >> np.uint64(k)) != 0, k + 1, bl)
    return 32 - bl


def _delta(codes, i, j):
    n = codes.shape[0]
    valid = (j >= 0) & (j <= n - 1)
    jj = np.clip(j, 0, n - 1)
    x = codes[i].astype(np.uint64) ^ codes[jj].astype(np.uint64)
    same = x == 0
    ix = (i ^ jj).astype(np.uint64)
    r = np.where(same, 32 + clz32(np.where(same, ix, 1)), clz32(np.where(same, 1, x)))
    return np.where(valid, r, -1)


def karras_tree(sorted_codes):
    """Build the tree for n sorted codes.

    Returns dict: child [2][n-1] int32 (left, right), parent_internal [n-1]
    (root: -1), parent_leaf [n], lo/hi [n-1] (leaf range of each internal node),
    split [n-1] (gamma).  n == 1: no internal nodes, the root is leaf 0.
    """
    codes = np.asarray(sorted_codes, dtype=np.uint32)
    n = codes.shape[0]
    m = max(n - 1, 0)
    out = {
        "child": np.zeros((2, m), np.int32),
        "parent_internal": np.full(m, -1, np.int32),
        "parent_leaf": np.full(n, -1, np.int32),
        "lo": np.zeros(m, np.int32),
        "hi": np.zeros(m, np.int32),
        "split": np.zeros(m, np.int32),
    }
    if n <= 1:
        return out
    i = np.arange(m, dtype=np.int64)
    # direction of the range: towards the neighbour sharing the longer prefix
    d = np.sign(_delta(codes, i, i + 1) - _delta(codes, i, i - 1)).astype(np.int64)
    dmin = _delta(codes, i, i - d)
    # exponential search for an upper bound of the range length
    lmax = np.full(m, 2, np.int64)
    act = _delta(codes, i, i + lmax * d) > dmin
    while act.any():
        lmax = np.where(act, lmax * 2, lmax)
        act = act & (_delta(codes, i, i + lmax * d) > dmin)
    # binary search for the other end
    l = np.zeros(m, np.int64)
    t = lmax // 2
    while (t >= 1).any():
        ok = (t >= 1) & (_delta(codes, i, i + (l + t) * d) > dmin)
        l = np.where(ok, l + t, l)
        t = t // 2
    j = i + l * d
    dnode = _delta(codes, i, j)
    # binary search for the split: t = ceil(l/2), ceil(l/4), ..., 1
    s = np.zeros(m, np.int64)
    div = 2
    act = np.ones(m, bool)
    while act.any():
        t = (l + div - 1) // div
        ok = act & (_delta(codes, i, i + (s + t) * d) > dnode)
        s = np.where(ok, s + t, s)
        act = act & (t > 1)
        div *= 2
    gamma = i + s * d + np.minimum(d, 0)
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    left = np.where(lo == gamma, ~gamma, gamma)
    right = np.where(hi == gamma + 1, ~(gamma + 1), gamma + 1)
    out["child"] = np.stack([left, right]).astype(np.int32)
    out["lo"], out["hi"], out["split"] = lo.astype(np.int32), hi.astype(np.int32), gamma.astype(np.int32)
    for c in (left, right):
        internal = c >= 0
        out["parent_internal"][c[internal]] = i[internal]
        out["parent_leaf"][~c[~internal]] = i[~internal]
    return out


def leaf_boxes(verts, faces, perm):
    """Leaf boxes [n,6] (lo xyz, hi xyz) in sorted order; faces None means point primitives."""
    V = np.asarray(verts, dtype=np.float64)
    perm = np.asarray(perm, dtype=np.int64)
    if faces is None:
        p = V[:, perm].T
        return np.concatenate([p, p], axis=1)
    F = np.asarray(faces).astype(np.int64)[:, perm]
    a, b, c = V[:, F[0]].T, V[:, F[1]].T, V[:, F[2]].T
    return np.concatenate([np.minimum(np.minimum(a, b), c), np.maximum(np.maximum(a, b), c)], axis=1)


def node_depths(tree, n):
    """Depth of every internal node (root 0), by breadth-first expansion."""
    m = max(n - 1, 0)
    depth = np.full(m, -1, np.int64)
    if m == 0:
        return depth
    front = np.array([0])
    dcur = 0
    while front.size:
        depth[front] = dcur
        ch = tree["child"][:, front].reshape(-1)
        front = ch[ch >= 0]
        dcur += 1
    return depth


def refit(tree, leaf_box):
    """Internal boxes [n-1,6]: union of the children's boxes, deepest level first."""
    n = leaf_box.shape[0]
    m = max(n - 1, 0)
    box = np.zeros((m, 6))
    if m == 0:
        return box
    depth = node_depths(tree, n)

    def child_box(c):
        out = np.empty((c.size, 6))
        internal = c >= 0
        out[internal] = box[c[internal]]
        out[~internal] = leaf_box[~c[~internal]]
        return out

    for dl in range(depth.max(), -1, -1):
        nodes = np.nonzero(depth == dl)[0]
        a = child_box(tree["child"][0, nodes])
        b = child_box(tree["child"][1, nodes])
        box[nodes, :3] = np.minimum(a[:, :3], b[:, :3])
        box[nodes, 3:] = np.maximum(a[:, 3:], b[:, 3:])
    return box


def build(verts, faces):
    """Whole build: codes, stable sort, tree, leaf and internal boxes (faces None: points)."""
    from .morton import morton_codes, sort_codes
    codes = morton_codes(verts, faces)
    scodes, perm = sort_codes(codes)
    tree = karras_tree(scodes)
    lb = leaf_boxes(verts, faces, perm)
    ib = refit(tree, lb)
    root = lb[0] if lb.shape[0] == 1 else (ib[0] if ib.shape[0] else np.zeros(6))
    return {"codes": codes, "sorted_codes": scodes, "perm": perm, "tree": tree,
            "leaf_box": lb, "internal_box": ib, "root_box": root}
