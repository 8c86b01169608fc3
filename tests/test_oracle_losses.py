"""Pins of the oracle's losses, gradients and Adam (CPU only)."""

import numpy as np
import pytest
import torch

from oracle import losses as olo
from oracle import gaussians as og
from oracle import adam as oa


def test_chamfer_closed_forms():
    rng = np.random.default_rng(30)
    A = rng.random((3, 400))
    cd, *_ = olo.chamfer(A, A)
    assert cd == 0.0
    # minimum pair spacing bounds the shift that keeps every nearest neighbour
    from scipy.spatial import cKDTree
    dmin = cKDTree(A.T).query(A.T, k=2)[0][:, 1].min()
    t = np.array([[0.3], [-0.2], [0.1]])
    t *= 0.25 * dmin / np.linalg.norm(t)
    cd, *_ = olo.chamfer(A, A + t)
    assert cd == pytest.approx(2 * (t ** 2).sum(), rel=1e-9)


def _fd_subset():
    from synth import make_config
    sc = make_config(4, small=True)
    return sc.verts0.astype(np.float64), sc.faces, sc.binding, sc.extra["targets"].astype(np.float64)


def _loss_and_argmins(V, F, b, Y):
    L, aux = olo.template_loss(V, F, b, Y)
    return L, (aux["rec"]["face"], aux["nn_ab"], aux["nn_ba"])


def test_template_gradient_vs_central_differences():
    V, F, b, Y = _fd_subset()
    assert F.shape[1] == 500 and b["face"].size == 1250 and Y.shape[1] == 2000
    L, g, aux = olo.template_loss_grad(V, F, b, Y)
    Lext = np.ptp(V, axis=1).max()
    h = 1e-6 * Lext
    rng = np.random.default_rng(31)
    coords = [(int(rng.integers(0, 3)), int(v)) for v in rng.choice(V.shape[1], 40, replace=False)]
    base = (aux["rec"]["face"], aux["nn_ab"], aux["nn_ba"])
    an, fd = [], []
    for ax, vi in coords:
        vals, same = [], True
        for s in (h, -h):
            Vs = V.copy()
            Vs[ax, vi] += s
            Ls, am = _loss_and_argmins(Vs, F, b, Y)
            vals.append(Ls)
            same &= all(np.array_equal(x, y) for x, y in zip(am, base))
        if same:   # coordinates whose +-h changes an argmin are excluded
            fd.append((vals[0] - vals[1]) / (2 * h))
            an.append(g[ax, vi])
    assert len(fd) >= 20
    an, fd = np.array(an), np.array(fd)
    assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd)


def test_binding_vjp_vs_central_differences():
    rng = np.random.default_rng(32)
    from synth import uv_sphere
    xhat, f = uv_sphere(10, 5)
    V = (xhat * (1 + 0.2 * rng.random((xhat.shape[0], 1)))).T.copy()
    F = f.T
    G = 300
    b = {"face": rng.integers(0, F.shape[1], G), "bary": rng.dirichlet([1, 1, 1], G).T[1:],
         "q_local": rng.normal(size=(4, G)), "log_scale": rng.normal(-1, 0.3, (3, G))}
    off = rng.normal(0, 0.05, G)
    gm, gR, gc = rng.normal(size=(3, G)), rng.normal(size=(G, 3, 3)), rng.normal(size=(6, G))

    def scalar(X):
        o = og.repose(X, F, b, offset=off)
        return (gm * o["mean"]).sum() + (gR * o["rot"]).sum() + (gc * o["cov"]).sum()

    g = olo.binding_vjp(V, F, b, gm, gR, gc, offset=off)
    coords = [(ax, vi) for vi in range(0, V.shape[1], 3) for ax in range(3)]
    fd = olo.central_difference(scalar, V, coords, 1e-6)
    an = np.array([g[ax, vi] for ax, vi in coords])
    assert np.linalg.norm(an - fd) <= 1e-7 * np.linalg.norm(fd)


def test_point_to_mesh_gradient_translation():
    # moving the mesh and the targets together leaves P unchanged, so dP/dV summed
    # over vertices equals minus the gradient w.r.t. a rigid shift of the targets
    V, F, b, Y = _fd_subset()
    P, rec = olo.point_to_mesh(V, F, Y)
    g = olo.point_to_mesh_grad(V, F, Y, rec)
    gy = 2.0 * (Y - rec["point"]).sum(1) / Y.shape[1]
    np.testing.assert_allclose(g.sum(1), -gy, rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(33)
    theta = rng.normal(size=(3, 50))
    p = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for step in range(1, 8):
        g = rng.normal(size=theta.shape)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = oa.adam_step(th, g, m, v, step, 1e-3)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)
