"""Seeded smooth shapes and motions of sphere-like templates.

* RadialShape: static radius field r(x) = 1 + sum_j a_j sin(k_j (d_j . x) + p_j) over
  the unit direction x (4 terms, a_j ~ U(0, 0.05), k_j ~ U(1, 3), d_j uniform on the
  sphere, p_j ~ U(0, 2 pi)).
* RadialMotion: time-varying radial offset u(x, t) = A sum_j sin(k_j (e_j . x) +
  2 pi n_j t / T + p_j), 3 terms, n_j ~ U(0.5, 2) cycles per sequence.
* VectorMotion: the same sinusoids along 3 random directions d_j (vector field).

Frames are evaluated in float64 and rounded once to float32.
"""

import numpy as np


def _unit_vectors(rng, n):
    x = rng.normal(size=(n, 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


class RadialShape:
    def __init__(self, rng, terms=4, amp=0.05):
        self.a = rng.uniform(0.0, amp, terms)
        self.k = rng.uniform(1.0, 3.0, terms)
        self.d = _unit_vectors(rng, terms)
        self.p = rng.uniform(0.0, 2.0 * np.pi, terms)

    def radius(self, xhat):
        arg = xhat @ self.d.T * self.k + self.p
        return 1.0 + (self.a * np.sin(arg)).sum(axis=-1)


class RadialMotion:
    def __init__(self, rng, n_frames, terms=3, amp=0.05):
        self.T = int(n_frames)
        self.amp = amp
        self.e = _unit_vectors(rng, terms)
        self.k = rng.uniform(1.0, 3.0, terms)
        self.nu = rng.uniform(0.5, 2.0, terms)
        self.p = rng.uniform(0.0, 2.0 * np.pi, terms)

    def offset(self, xhat, t):
        arg = xhat @ self.e.T * self.k + 2.0 * np.pi * self.nu * (t / self.T) + self.p
        return self.amp * np.sin(arg).sum(axis=-1)


class VectorMotion:
    def __init__(self, rng, n_frames, terms=3, amp=0.05):
        self.T = int(n_frames)
        self.amp = amp
        self.dirs = _unit_vectors(rng, terms)
        self.e = _unit_vectors(rng, terms)
        self.k = rng.uniform(1.0, 3.0, terms)
        self.nu = rng.uniform(0.5, 2.0, terms)
        self.p = rng.uniform(0.0, 2.0 * np.pi, terms)

    def displacement(self, x, t):
        arg = x @ self.e.T * self.k + 2.0 * np.pi * self.nu * (t / self.T) + self.p
        return self.amp * np.sin(arg) @ self.dirs


def radial_template(xhat, shape):
    """Template vertices r(x) * x for unit directions x (AoS float64)."""
    return xhat * shape.radius(xhat)[:, None]


def frames_radial(xhat, shape, motion, ts):
    """Frame store [T][3][V] float32: (r(x) + u(x, t)) x for each t in ts."""
    r0 = shape.radius(xhat)
    out = np.empty((len(ts), 3, xhat.shape[0]), np.float32)
    for i, t in enumerate(ts):
        r = r0 + motion.offset(xhat, float(t))
        out[i] = (xhat * r[:, None]).T.astype(np.float32)
    return out


def frames_vector(v0, motion, ts):
    """Frame store [T][3][V] float32: v0 + u(v0, t)."""
    out = np.empty((len(ts), 3, v0.shape[0]), np.float32)
    for i, t in enumerate(ts):
        out[i] = (v0 + motion.displacement(v0, float(t))).T.astype(np.float32)
    return out
