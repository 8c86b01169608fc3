"""mg_frame_update (copy, re-pose and refit in one launch) against the three separate
calls it fuses: the live buffer, every Gaussian output and every BVH byte the refit
writes are bitwise equal; a sample of means is also checked against the oracle."""

import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, dev, host, scale_of, assert_positions
from synth import make_config
from oracle import gaussians as og

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def _refit_bytes(bvh):
    """The bytes a refit writes: the node records, and the header's counts, status and
    root box (not its padding, which nothing writes)."""
    L = bvh.layout
    m = max(bvh.n - 1, 0)
    b = host(bvh.buf)
    hdr = b[:64].view(np.uint32)
    return b[L.off_nodes:L.off_nodes + 96 * m], np.concatenate([hdr[0:7], hdr[8:11]])


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_frame_update_equals_separate_calls(device, cfg):
    import paper_2606_00444_amd as mg
    sc = make_config(cfg)
    frames_np = sc.frames([0, 7, 33])
    frames = dev(frames_np, device)
    F = dev(sc.faces, device)
    b = {k: dev(v, device) for k, v in sc.binding.items()}
    V0 = dev(sc.verts0, device)
    bvh_a, bvh_b = mg.lbvh_build(V0, F), mg.lbvh_build(V0, F)
    live_a = torch.empty(3, sc.n_verts, device=device)
    live_b = torch.full((3, sc.n_verts), float("nan"), device=device)
    for k in (1, 2, 0):                      # consecutive frames through the same BVH
        print(f"frame update: config {cfg}, frame {k}", flush=True)
        mg.vertex_buffer_update(frames, k, live_a)
        ga = mg.mesh_gaussian_update(live_a, F, b["face"], b["bary"], b["q_local"], b["log_scale"], rot=True)
        mg.lbvh_refit(bvh_a, live_a)
        gb = mg.frame_update(frames, k, live_b, F, b["face"], b["bary"], b["q_local"], b["log_scale"], bvh_b,
                             rot=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(live_b).view(np.uint32), host(live_a).view(np.uint32))
        for key in ("mean", "quat", "cov", "rot"):
            np.testing.assert_array_equal(host(gb[key]).view(np.uint32), host(ga[key]).view(np.uint32))
        na, ha = _refit_bytes(bvh_a)
        nb, hb = _refit_bytes(bvh_b)
        np.testing.assert_array_equal(nb, na)
        np.testing.assert_array_equal(hb, ha)
        assert int(host(bvh_b.buf[:16].view(torch.int32))[2]) == 0
    # a sample of the fused path's means against the float64 oracle (frame 0)
    rng = np.random.default_rng(cfg)
    idx = np.sort(rng.choice(sc.n_gauss, min(2000, sc.n_gauss), replace=False))
    sub = {k: np.asarray(sc.binding[k])[..., idx] for k in ("face", "bary", "q_local", "log_scale")}
    ref = og.repose(frames_np[0].astype(np.float64), sc.faces, sub)
    assert_positions(host(gb["mean"])[:, idx], ref["mean"], scale_of(frames_np[0]), "means")


def test_frame_update_without_gaussians(device):
    import paper_2606_00444_amd as mg
    sc = make_config(1)
    frames = dev(sc.frames([0, 5]), device)
    F = dev(sc.faces, device)
    V0 = dev(sc.verts0, device)
    bvh_a, bvh_b = mg.lbvh_build(V0, F), mg.lbvh_build(V0, F)
    live = torch.empty(3, sc.n_verts, device=device)
    empty_i = torch.empty(0, dtype=torch.int32, device=device)
    e2, e4, e3 = (torch.empty(r, 0, device=device) for r in (2, 4, 3))
    mg.frame_update(frames, 1, live, F, empty_i, e2, e4, e3, bvh_b)
    mg.lbvh_refit(bvh_a, frames[1].contiguous())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(live), host(frames[1]))
    np.testing.assert_array_equal(_refit_bytes(bvh_b)[0], _refit_bytes(bvh_a)[0])


def test_frame_update_2048_leaf_subtrees(device):
    """A mesh of more than 524,288 faces (the 1M-face split target of the large
    configuration as a fixed template): 2048-leaf subtrees, four nodes per thread.
    Fused against separate calls, bitwise, on a displaced copy of the vertices."""
    import paper_2606_00444_amd as mg
    from synth.gaussians import draw_binding
    sc = make_config(5)
    v, f = sc.target(3)
    assert f.shape[1] > 524288
    rng = np.random.default_rng(11)
    b_np = draw_binding(rng, v.T.astype(np.float64), f.T, n_gauss=200_000)
    L = scale_of(v)
    frames_np = np.stack([v, v + (rng.normal(size=v.shape) * 1e-3 * L).astype(np.float32)])
    frames = dev(frames_np, device)
    F = dev(f, device)
    b = {k: dev(b_np[k], device) for k in ("face", "bary", "q_local", "log_scale")}
    bvh_a, bvh_b = mg.lbvh_build(frames[0].contiguous(), F), mg.lbvh_build(frames[0].contiguous(), F)
    live_a = torch.empty(3, v.shape[1], device=device)
    live_b = torch.empty(3, v.shape[1], device=device)
    print("frame update: 1M-face mesh, frame 1", flush=True)
    mg.vertex_buffer_update(frames, 1, live_a)
    ga = mg.mesh_gaussian_update(live_a, F, b["face"], b["bary"], b["q_local"], b["log_scale"])
    mg.lbvh_refit(bvh_a, live_a)
    gb = mg.frame_update(frames, 1, live_b, F, b["face"], b["bary"], b["q_local"], b["log_scale"], bvh_b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(live_b).view(np.uint32), host(live_a).view(np.uint32))
    for key in ("mean", "quat", "cov"):
        np.testing.assert_array_equal(host(gb[key]).view(np.uint32), host(ga[key]).view(np.uint32))
    na, ha = _refit_bytes(bvh_a)
    nb, hb = _refit_bytes(bvh_b)
    np.testing.assert_array_equal(nb, na)
    np.testing.assert_array_equal(hb, ha)
    assert int(host(bvh_b.buf[:16].view(torch.int32))[2]) == 0
