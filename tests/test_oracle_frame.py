"""The oracle's frame selection and vertex-buffer update against hand-worked values
(paper Sec. 3.3 MaGS paragraph: k = floor(t f_recon); Sec. 3.4 per-frame step 2:
the O(N_v) copy of frame k into the live vertex buffer)."""

import json
import os

import numpy as np
import pytest

from oracle import frame as of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "frame_index.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: c["why"][:40])
def test_frame_index_worked_cases(case):
    want = case.get("clamped_k", case["k"])
    got = of.frame_index(case["step"], case["num"], case["den"], case["f_sim"], case["n_frames"])
    assert isinstance(got, int) and got == want
    # the unclamped value is the floor of the exact rational t * f_recon
    big = of.frame_index(case["step"], case["num"], case["den"], case["f_sim"], 1 << 62)
    assert big == case["k"]


@pytest.mark.parametrize("case", _golden()["invalid"])
def test_frame_index_rejects_invalid(case):
    with pytest.raises(ValueError):
        of.frame_index(case["step"], case["num"], case["den"], case["f_sim"], case["n_frames"])


def test_frame_index_is_monotone_and_steps_by_the_rate():
    # at f_recon = f_sim / 2 every frame is held for exactly two simulation steps
    ks = [of.frame_index(s, 30, 1, 60, 1000) for s in range(200)]
    assert ks == [s // 2 for s in range(200)]
    # at a rate ratio of 24000/1001 over 60 the frame advances by 0 or 1 per step, and
    # after 60 * 1001 steps exactly 24000 frames have passed
    ks = [of.frame_index(s, 24000, 1001, 60, 10 ** 9) for s in range(0, 60 * 1001 + 1)]
    d = np.diff(ks)
    assert set(d.tolist()) <= {0, 1} and ks[-1] == 24000


def test_vertex_buffer_update_is_a_bitwise_copy_of_frame_k():
    rng = np.random.default_rng(11)
    T, V = 5, 37
    frames = rng.normal(size=(T, 3, V)).astype(np.float32)
    # awkward float32 payloads: signed zero, a quiet NaN with a payload, a subnormal, infinities
    special = np.array([0x80000000, 0x7FC01234, 0x00000001, 0x7F800000, 0xFF800000], dtype=np.uint32)
    frames[3, 1, :5] = special.view(np.float32)
    for k in range(T):
        live = of.vertex_buffer_update(frames, k)
        assert live.shape == (3, V) and live.dtype == np.float32
        assert live.tobytes() == frames[k].tobytes()
    # the live buffer is a copy: writing it leaves the frame store unchanged
    keep = frames.copy()
    live = of.vertex_buffer_update(frames, 2)
    live[:] = 0
    assert frames.tobytes() == keep.tobytes()
