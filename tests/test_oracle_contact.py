"""Pins of the sphere-mesh contact step oracle (collision response)."""

import numpy as np

from oracle import contact as oct_

# a large square floor at z = 0 (normal +z), two triangles
FLOOR_V = np.array([[-10, -10, 0], [10, -10, 0], [10, 10, 0], [-10, 10, 0]], dtype=np.float64).T
FLOOR_F = np.array([[0, 1, 2], [0, 2, 3]]).T
G = np.array([0.0, 0.0, -9.8])


def test_free_flight_is_semi_implicit_euler():
    x0 = np.array([[0.0], [0.0], [5.0]])
    v0 = np.array([[1.0], [0.5], [0.0]])
    dt, n = 0.01, 30
    x, v = x0, v0
    for _ in range(n):
        x, v, c = oct_.step(x, v, FLOOR_V, FLOOR_F, dt, G, 0.1, 0.5)
        assert not c.any()
    # closed form: v_n = v0 + n g dt, x_n = x0 + dt (n v0 + g dt n(n+1)/2)
    np.testing.assert_allclose(v[:, 0], v0[:, 0] + n * G * dt, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x[:, 0], x0[:, 0] + dt * (n * v0[:, 0] + G * dt * n * (n + 1) / 2), rtol=1e-12,
                               atol=1e-12)


def test_resting_and_bouncing_on_the_floor():
    r = 0.25
    # inelastic: lands and rests with its centre exactly at height r, vertical velocity 0
    x, v = np.array([[0.3], [0.2], [1.0]]), np.zeros((3, 1))
    for _ in range(200):
        x, v, c = oct_.step(x, v, FLOOR_V, FLOOR_F, 0.01, G, r, 0.0)
    assert c[0]
    np.testing.assert_allclose(x[:, 0], [0.3, 0.2, r], rtol=0, atol=1e-12)
    assert v[2, 0] == 0.0
    # elastic: a sphere arriving at -3 m/s leaves at +3 m/s (minus this step's gravity kick)
    x, v = np.array([[0.0], [0.0], [r + 0.01]]), np.array([[0.0], [0.0], [-3.0]])
    x, v, c = oct_.step(x, v, FLOOR_V, FLOOR_F, 0.01, np.zeros(3), r, 1.0)
    assert c[0]
    np.testing.assert_allclose(v[:, 0], [0.0, 0.0, 3.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[:, 0], [0.0, 0.0, r], rtol=0, atol=1e-12)


def test_tunnelled_centre_is_pushed_out_along_the_face_normal():
    r = 0.1
    x, v = np.array([[1.0], [1.0], [-0.05]]), np.array([[0.0], [0.0], [-1.0]])
    x1, v1, c = oct_.step(x, v, FLOOR_V, FLOOR_F, 0.01, np.zeros(3), r, 0.0)
    assert c[0]
    np.testing.assert_allclose(x1[:, 0], [1.0, 1.0, r], rtol=0, atol=1e-12)
    np.testing.assert_allclose(v1[:, 0], [0.0, 0.0, 0.0], rtol=0, atol=1e-12)


def test_edge_contact_normal_points_from_the_edge():
    # a sphere beside the floor's edge x = 10 at height 0.05: contact normal from the edge
    r = 0.2
    x, v = np.array([[10.1], [0.0], [0.05]]), np.array([[-1.0], [0.0], [0.0]])
    x1, v1, c = oct_.step(x, v, FLOOR_V, FLOOR_F, 0.0, np.zeros(3), r, 0.0)
    assert c[0]
    d = np.array([0.1, 0.0, 0.05])
    nh = d / np.linalg.norm(d)
    np.testing.assert_allclose(x1[:, 0], np.array([10.0, 0.0, 0.0]) + r * nh, rtol=0, atol=1e-12)
    np.testing.assert_allclose((v1[:, 0] * nh).sum(), 0.0, atol=1e-12)      # normal velocity removed
