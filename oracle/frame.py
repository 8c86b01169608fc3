"""Frame selection and vertex-buffer update (Sec. 3.3 MaGS paragraph; Sec. 3.4 steps 1-2).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

import numpy as np


def frame_index(step, f_recon_num, f_recon_den, f_sim, n_frames):
    """k = floor(t * f_recon) with t = step / f_sim and f_recon = num / den, clamped to n_frames - 1.

    The paper states k = floor(t f_recon); it does not say what happens past the
    last frame or how t is represented.  Reading: integer arithmetic (no float
    rounding) and clamping (no wrap-around).
    """
    if step < 0 or f_recon_num < 0 or f_recon_den <= 0 or f_sim <= 0 or n_frames <= 0:
        raise ValueError("invalid frame-index arguments")
    k = (int(step) * int(f_recon_num)) // (int(f_sim) * int(f_recon_den))
    return min(k, int(n_frames) - 1)


def vertex_buffer_update(frames, k):
    """V_live = V_k: a bitwise copy of frame k of a [T][3][V] frame store."""
    return np.array(frames[k], copy=True)
