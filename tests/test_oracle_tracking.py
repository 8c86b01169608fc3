"""Pins of the temporal-tracking oracle (Strategy 1, Sec. 3.3, Eq. 1)."""

import numpy as np

from oracle import tracking as otr
from oracle import closest as oc
from synth.meshes import icosphere


def _square(z=0.0, x0=0.0):
    """Unit square [x0, x0+1] x [0, 1] at height z as two triangles (SoA)."""
    v = np.array([[x0, 0, z], [x0 + 1, 0, z], [x0 + 1, 1, z], [x0, 1, z]], dtype=np.float64).T
    f = np.array([[0, 1, 2], [0, 2, 3]]).T
    return v, f


def test_static_sequence_is_the_identity():
    v, f = icosphere(1)
    V, F = v.T.astype(np.float64), f.T
    tr = otr.track(V, [(V, F)] * 7, every=3)
    for t in range(7):
        np.testing.assert_array_equal(tr[t], V)     # a vertex's closest point is itself


def test_plane_moving_along_its_normal():
    # points on the plane follow it (to the rounding of rebuilding the closest point
    # from its barycentrics); template projection agrees, so the re-anchoring blend
    # changes nothing
    rng = np.random.default_rng(0)
    P = np.vstack([rng.random((2, 40)), np.zeros((1, 40))])
    targets = [_square(z=0.25 * t) for t in range(9)]
    tr = otr.track(P, targets, every=4)
    for t in range(9):
        np.testing.assert_allclose(tr[t][:2], P[:2], rtol=0, atol=1e-14)
        np.testing.assert_allclose(tr[t][2], np.full(40, 0.25 * t), rtol=0, atol=1e-14)


def test_reanchor_blend_worked_example():
    # the square slides +x by 0.5 per frame; points left behind are clamped to its
    # left edge by tracking, while the template projection clamps the template's
    # points: at the re-anchoring frame the result is 0.8 tracked + 0.2 projection
    P = np.array([[0.1, 0.6, 0.9], [0.5, 0.5, 0.5], [0.0, 0.0, 0.0]])
    targets = [_square(x0=0.5 * t) for t in range(3)]
    tr = otr.track(P, targets, every=2)
    # frame 1 (square [0.5, 1.5]): x = 0.5, 0.6, 0.9
    np.testing.assert_allclose(tr[1][0], [0.5, 0.6, 0.9], rtol=0, atol=1e-14)
    # frame 2 (square [1, 2]): tracked x = 1, 1, 1; template projection x = 1, 1, 1
    np.testing.assert_allclose(tr[2][0], [1.0, 1.0, 1.0], rtol=0, atol=1e-14)
    # blend weights: with every=1 and w_track=0 each frame is the template projection (Eq. 2)
    tr0 = otr.track(P, targets, every=1, w_track=0.0)
    for t in range(1, 3):
        np.testing.assert_array_equal(tr0[t], oc.template_projection(P, *targets[t])[0])
    # with w_track=1 re-anchoring is a no-op: plain tracking
    tr1 = otr.track(P, targets, every=1, w_track=1.0)
    np.testing.assert_array_equal(tr1, otr.track(P, targets, every=0))


def test_blend_of_distinct_tracks():
    # tracked and template-projected points differ: a point carried to the left edge
    # at frame 1 (x = 0.5) and the template point x = 0.1 both clamp to x = 1 at
    # frame 2 on [1, 2] ... use a frame where they differ: the square returns to
    # [0.5, 1.5] at frame 2, so tracking keeps x = 0.5 and projection gives x = 0.5;
    # with the square at [0.3, 1.3], tracking keeps 0.5 and projection gives 0.3
    P = np.array([[0.1], [0.5], [0.0]])
    targets = [_square(x0=0.0), _square(x0=0.5), _square(x0=0.3)]
    tr = otr.track(P, targets, every=2, w_track=0.8)
    np.testing.assert_allclose(tr[2][0], [0.8 * 0.5 + 0.2 * 0.3], rtol=0, atol=1e-14)
    np.testing.assert_allclose(tr[2][1:], [[0.5], [0.0]], rtol=0, atol=1e-14)


def test_knn_variant_reduces_to_closest_and_keeps_static_points():
    v, f = icosphere(1)
    V, F = v.T.astype(np.float64), f.T
    targets = [(V, F)] * 4
    # vertices are exact hits: with any k the track stays put
    np.testing.assert_array_equal(otr.track(V, targets, every=2, k=4), np.stack([V] * 4))
    # k = 1 is the closest-point track
    P = 0.9 * V
    tv, tf = _square(z=0.1)
    a = otr.track(P[:, :10], [(tv, tf)] * 3, every=2, k=1)
    b = otr.track(P[:, :10], [(tv, tf)] * 3, every=2)
    np.testing.assert_array_equal(a, b)
