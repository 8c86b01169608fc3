"""The seeded input generators: sizes, determinism, closed outward-facing surfaces (CPU only)."""

import numpy as np
import pytest

from synth import icosphere, uv_sphere, make_config, marching_tetrahedra


def _euler_and_volume(v, f):
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e.sort(axis=1)
    n_e = np.unique(e[:, 0] * (v.shape[0] + 1) + e[:, 1]).size
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    vol = (a * np.cross(b, c)).sum() / 6.0
    return v.shape[0] - n_e + f.shape[0], vol


def test_template_sizes():
    v, f = icosphere(4)
    assert v.shape == (2562, 3) and f.shape == (5120, 3)
    for (nl, nr, nv, nf) in [(200, 100, 20002, 40000), (1000, 250, 250002, 500000), (25, 10, 252, 500)]:
        v, f = uv_sphere(nl, nr)
        assert v.shape[0] == nv and f.shape[0] == nf


@pytest.mark.parametrize("mesh", ["ico", "uv", "mt"])
def test_closed_and_outward(mesh):
    if mesh == "ico":
        v, f = icosphere(3)
    elif mesh == "uv":
        v, f = uv_sphere(30, 12)
    else:
        g = np.linspace(-1.4, 1.4, 31)
        x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1)
        phi = np.linalg.norm(x, axis=-1) - 1.0
        v, f = marching_tetrahedra(phi, np.array([-1.4] * 3), g[1] - g[0])
    chi, vol = _euler_and_volume(v, f)
    assert chi == 2
    assert vol == pytest.approx(4.0 / 3.0 * np.pi, rel=0.05)


def test_configs_deterministic_and_sized():
    a = make_config(1)
    b = make_config(1)
    np.testing.assert_array_equal(a.queries, b.queries)
    np.testing.assert_array_equal(a.binding["q_local"], b.binding["q_local"])
    assert a.n_verts == 2562 and a.n_faces == 5120 and a.n_gauss == 30720 and a.queries.shape == (3, 10000)
    c2 = make_config(2)
    assert c2.n_verts == 20002 and c2.n_faces == 40000 and c2.n_gauss == 100000
    assert c2.queries.shape == (3, 50000)
    tv, tf = c2.target(0)
    assert 30000 <= tf.shape[1] <= 60000
    assert tf.min() >= 0 and tf.max() < tv.shape[1]
    b = c2.binding
    assert (np.diff(b["face"]) >= 0).all()
    np.testing.assert_array_equal(np.bincount(b["face"], minlength=40000), np.diff(b["face_offsets"]))
    q = b["q_local"].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(q, axis=0), 1.0, atol=1e-6)
    assert (b["bary"] >= 0).all() and (b["bary"].sum(0) <= 1.0 + 1e-6).all()


def test_split_target_counts():
    sc = make_config(5, small=True)
    tv, tf = sc.target(3)
    assert tf.shape[1] == 2 * sc.n_faces and tv.shape[1] == sc.n_verts + sc.n_faces
