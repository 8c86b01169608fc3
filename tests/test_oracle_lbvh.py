"""Pins of the oracle's Morton codes, stable sort, Karras tree and refit (CPU only)."""

import json
import os
import struct

import numpy as np
import pytest

from oracle import morton as om
from oracle import lbvh as ol

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f32(x):
    """Round a Python float to binary32 (round-to-nearest-even) and back."""
    return struct.unpack("f", struct.pack("f", x))[0]


def morton_scalar(verts, faces):
    """Per-element binary32 definition with explicit rounding of every operation.

    Each +, -, *, / of two binary32 values is computed in binary64 and rounded
    once to binary32; for these operations that equals the correctly rounded
    binary32 result (53 >= 2 * 24 + 2), so this is an independent route to
    the definition.  Interleave by string concatenation of bits.
    """
    V = np.asarray(verts, dtype=np.float32).astype(np.float64)
    n = faces.shape[1] if faces is not None else V.shape[1]
    s = np.empty((3, n))
    for i in range(n):
        for ax in range(3):
            if faces is None:
                s[ax, i] = V[ax, i]
            else:
                a, b, c = (V[ax, faces[k, i]] for k in range(3))
                s[ax, i] = f32(f32(a + b) + c)
    codes = []
    lo = [min(s[ax]) for ax in range(3)]
    hi = [max(s[ax]) for ax in range(3)]
    scale = [f32(1024.0 / f32(hi[ax] - lo[ax])) if hi[ax] > lo[ax] else 0.0 for ax in range(3)]
    for i in range(n):
        bits = []
        for ax in range(3):
            x = f32(f32(s[ax, i] - lo[ax]) * scale[ax])
            bits.append(format(min(1023, int(x)), "010b"))
        codes.append(int("".join(bits[0][k] + bits[1][k] + bits[2][k] for k in range(10)), 2))
    return np.array(codes, dtype=np.uint32)


def test_morton_binary32_definition():
    rng = np.random.default_rng(10)
    V = (rng.normal(size=(3, 200)) * np.array([[1.0], [0.01], [100.0]])).astype(np.float32)
    F = rng.integers(0, 200, size=(3, 300))
    np.testing.assert_array_equal(om.morton_codes(V, F), morton_scalar(V, F))
    P = rng.random(size=(3, 150)).astype(np.float32)
    np.testing.assert_array_equal(om.morton_codes(P, None), morton_scalar(P, None))


def test_morton_special_cases():
    # all centroids coincident: every code 0
    V = np.ones((3, 3), np.float32)
    F = np.array([[0, 1], [1, 2], [2, 0]])
    np.testing.assert_array_equal(om.morton_codes(V, F), 0)
    # planar mesh (z == 0): z bits all zero
    rng = np.random.default_rng(11)
    V = rng.random((3, 50)).astype(np.float32)
    V[2] = 0
    F = rng.integers(0, 50, size=(3, 40))
    c = om.morton_codes(V, F)
    zmask = sum(1 << (3 * i) for i in range(10))
    assert (c & np.uint32(zmask) == 0).all()
    # the primitive at the upper bound lands in cell 1023 on every axis
    P = np.array([[0.0, 1.0, 0.5], [0.0, 1.0, 0.25], [0.0, 1.0, 0.75]], np.float32)
    q, _, _ = om.quantize(om.centroid_sums(P, None))
    assert list(q[:, 1]) == [1023, 1023, 1023]
    assert list(q[:, 0]) == [0, 0, 0]
    assert list(q[:, 2]) == [512, 256, 768]
    assert om.morton_codes(P, None)[1] == (1 << 30) - 1


def test_fp64_boundary_ties_are_rare():
    from synth import make_config
    sc = make_config(2, small=True)
    q32, _, _ = om.quantize(om.centroid_sums(sc.verts0, sc.faces))
    q64 = om.quantize_fp64(sc.verts0, sc.faces)
    diff = np.abs(q32.astype(np.int64) - q64.astype(np.int64))
    assert diff.max() <= 1
    assert (diff.sum(0) > 0).mean() < 0.01


def test_stable_sort():
    rng = np.random.default_rng(12)
    codes = rng.integers(0, 16, 500).astype(np.uint32)
    s, perm = om.sort_codes(codes)
    ref = sorted(range(500), key=lambda i: (codes[i], i))
    np.testing.assert_array_equal(perm, ref)
    np.testing.assert_array_equal(s, codes[ref])


def topdown_tree(codes):
    """Karras's tree from its definition, recursively (independent of the oracle's search).

    Key of leaf i = (code_i, i).  A range [a, b] splits after the last leaf g
    whose key shares more leading bits with key a than key b does; children are
    numbered g (left) and g + 1 (right), one-leaf ranges are leaves.
    """
    n = len(codes)
    key = [(int(codes[i]) << 32) | i for i in range(n)]

    def common(x, y):
        z = x ^ y
        return 64 - z.bit_length()

    left, right = [0] * (n - 1), [0] * (n - 1)
    lo, hi = [0] * (n - 1), [0] * (n - 1)
    stack = [(0, n - 1, 0)]
    while stack:
        a, b, idx = stack.pop()
        lo[idx], hi[idx] = a, b
        c = common(key[a], key[b])
        g = a
        for k in range(a, b):
            if common(key[a], key[k + 1]) > c:
                g = k + 1
        lref = ~g if g == a else g
        rref = ~(g + 1) if g + 1 == b else g + 1
        left[idx], right[idx] = lref, rref
        if g > a:
            stack.append((a, g, g))
        if g + 1 < b:
            stack.append((g + 1, b, g + 1))
    return np.array(left), np.array(right), np.array(lo), np.array(hi)


def test_karras_golden():
    gold = json.load(open(os.path.join(GOLD, "karras_8keys.json")))
    t = ol.karras_tree(np.array(gold["codes"], dtype=np.uint32))
    np.testing.assert_array_equal(t["child"][0], gold["child_left"])
    np.testing.assert_array_equal(t["child"][1], gold["child_right"])
    np.testing.assert_array_equal(t["lo"], gold["lo"])
    np.testing.assert_array_equal(t["hi"], gold["hi"])


@pytest.mark.parametrize("n,maxcode,seed", [(2, 4, 0), (3, 4, 1), (5, 2, 2), (17, 8, 3), (100, 50, 4),
                                            (700, 1 << 30, 5), (600, 3, 6), (64, 1, 7)])
def test_karras_matches_topdown(n, maxcode, seed):
    rng = np.random.default_rng(seed)
    codes = np.sort(rng.integers(0, maxcode, n).astype(np.uint32))
    t = ol.karras_tree(codes)
    l, r, lo, hi = topdown_tree(codes)
    np.testing.assert_array_equal(t["child"][0], l)
    np.testing.assert_array_equal(t["child"][1], r)
    np.testing.assert_array_equal(t["lo"], lo)
    np.testing.assert_array_equal(t["hi"], hi)


def _check_tree_invariants(t, n):
    m = n - 1
    # every node except the root has exactly one parent
    ch = t["child"].reshape(-1)
    internal = np.sort(ch[ch >= 0])
    leaves = np.sort(~ch[ch < 0])
    np.testing.assert_array_equal(internal, np.arange(1, m))
    np.testing.assert_array_equal(leaves, np.arange(n))
    assert t["parent_internal"][0] == -1
    # in-order traversal visits leaves 0..n-1; ranges are contiguous
    order = []
    stack = [0]
    while stack:
        c = stack.pop()
        if c < 0:
            order.append(~c)
            continue
        stack.append(t["child"][1, c])
        stack.append(t["child"][0, c])
    np.testing.assert_array_equal(order, np.arange(n))
    assert ol.node_depths(t, n).max() <= 30 + int(np.ceil(np.log2(n))) + 1


def test_tree_invariants_degenerate_keys():
    for codes in (np.zeros(1000, np.uint32), np.repeat(np.arange(10, dtype=np.uint32), 37)):
        t = ol.karras_tree(codes)
        _check_tree_invariants(t, codes.size)


def test_single_and_empty():
    t = ol.karras_tree(np.zeros(1, np.uint32))
    assert t["child"].shape == (2, 0)
    assert t["parent_leaf"][0] == -1
    t = ol.karras_tree(np.zeros(0, np.uint32))
    assert t["child"].shape == (2, 0)


def test_refit_definition_and_invariants():
    from synth import make_config
    sc = make_config(2, small=True)
    fr = sc.frames([17])[0]
    b = ol.build(sc.verts0, sc.faces)
    n = sc.n_faces
    _check_tree_invariants(b["tree"], n)
    lb = ol.leaf_boxes(fr, sc.faces, b["perm"])
    ib = ol.refit(b["tree"], lb)
    # each internal box is the union of all leaf boxes of its range (brute force)
    for i in range(0, n - 1, 7):
        a, z = b["tree"]["lo"][i], b["tree"]["hi"][i]
        np.testing.assert_array_equal(ib[i, :3], lb[a:z + 1, :3].min(0))
        np.testing.assert_array_equal(ib[i, 3:], lb[a:z + 1, 3:].max(0))
    # root equals the mesh's bounding box, and the root of a fresh build of the same frame
    V = fr.astype(np.float64)
    used = np.unique(sc.faces)
    np.testing.assert_array_equal(ib[0, :3], V[:, used].min(1))
    np.testing.assert_array_equal(ib[0, 3:], V[:, used].max(1))
    fresh = ol.build(fr, sc.faces)
    np.testing.assert_array_equal(fresh["root_box"], ib[0])
    # refit on the rest pose reproduces the build's boxes; refit is idempotent
    np.testing.assert_array_equal(ol.refit(b["tree"], ol.leaf_boxes(sc.verts0, sc.faces, b["perm"])), b["internal_box"])
    np.testing.assert_array_equal(ol.refit(b["tree"], lb), ib)
    # enclosure: every child box inside its parent
    for side in (0, 1):
        c = b["tree"]["child"][side]
        cb = np.where((c >= 0)[:, None], ib[np.maximum(c, 0)], lb[np.maximum(~c, 0)])
        assert (cb[:, :3] >= ib[:, :3]).all() and (cb[:, 3:] <= ib[:, 3:]).all()
