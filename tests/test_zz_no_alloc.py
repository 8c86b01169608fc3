"""mg_lbvh_build_static (sort scratch in a static device array) against mg_lbvh_build
(caller workspace): the two BVH buffers are equal byte for byte, over two calls in
a row whose second builds a smaller tree on the scratch the first one left."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, dev, host
from paper_2606_00444_amd._lib import LbvhHeader
from synth import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def device():
    return need_gpu()


def _zeroed(mg, n, kind, device):
    # zero-filled buffers: bytes no build writes (padding) compare equal too
    return mg.LBVH(n, kind, device, buf=torch.zeros(mg.lbvh_bytes(n, kind), dtype=torch.uint8, device=device))


def _sec(b, L, name, count, dtype=np.int32):
    off = getattr(L, "off_" + name)
    return b[off:off + count * np.dtype(dtype).itemsize].view(dtype)


def _canonical(b, L, n):
    """The order-free content of the top-node and subtree lists.  Both are filled
    through atomic counters, so their order (and the indices that point into them)
    may differ between any two builds; what is unique is each top node's two
    children (a top node, or a subtree with its extent and deposited summary)."""
    hdr = LbvhHeader.from_buffer_copy(b[:ctypes.sizeof(LbvhHeader)].tobytes())
    n_top, n_sub = hdr.n_top, hdr.n_sub
    top = _sec(b, L, "top_nodes", n)[:n_top]
    tch = _sec(b, L, "top_child", 2 * n).reshape(2, n)
    sub = _sec(b, L, "subtrees", 3 * n).reshape(3, n)[:, :n_sub]
    dep = _sec(b, L, "deposits", 12 * n, np.float32).reshape(n, 12)[:n_sub].view(np.uint32)
    aux = _sec(b, L, "node_aux", max(n - 1, 0))
    # node_aux: -1 off the top, else the node's index in top_nodes
    on_top = np.flatnonzero(aux >= 0)
    assert (top[aux[on_top]] == on_top).all()

    def child(c):
        if c >= 0:
            return ("top", int(top[c]))
        k = ~c
        return ("sub", int(sub[0, k]), int(sub[1, k]), int(sub[2, k]), dep[k].tobytes())

    tops = {int(t): (child(int(tch[0, i])), child(int(tch[1, i]))) for i, t in enumerate(top)}
    subs = sorted((int(sub[0, k]), int(sub[1, k]), int(sub[2, k])) for k in range(n_sub))
    return np.sort(on_top), tops, subs


def _compare(mg, ref, got):
    """Byte for byte outside the lists filled through atomic counters (and the
    top-phase scratch, whose dummy slots hold whatever the losing lanes of a join
    wrote); those lists compare in order-free form."""
    L, n = ref.layout, ref.n
    a, b = host(ref.buf), host(got.buf)
    for lo, hi in ((0, L.off_node_aux), (L.off_child, L.off_top_nodes), (L.off_inv_prim, L.total_bytes)):
        diff = np.flatnonzero(a[lo:hi] != b[lo:hi])
        assert diff.size == 0, f"{diff.size} bytes differ in [{lo}, {hi}), first at {lo + diff[0]}"
    ca, cb = _canonical(a, L, n), _canonical(b, L, n)
    np.testing.assert_array_equal(ca[0], cb[0])
    assert ca[1] == cb[1]
    assert ca[2] == cb[2]
    assert LbvhHeader.from_buffer_copy(b[:ctypes.sizeof(LbvhHeader)].tobytes()).status == 0


def _pair(mg, verts, faces, device):
    kind = mg.MG_PRIM_POINTS if faces is None else mg.MG_PRIM_TRIANGLES
    n = verts.shape[1] if faces is None else faces.shape[1]
    V = dev(verts, device)
    Fd = None if faces is None else dev(faces, device)
    ref = mg.lbvh_build(V, Fd, bvh=_zeroed(mg, n, kind, device))
    got = mg.lbvh_build_static(V, Fd, _zeroed(mg, n, kind, device))
    torch.cuda.synchronize()
    _compare(mg, ref, got)


def test_static_build_matches_workspace_build(device):
    import paper_2606_00444_amd as mg
    big = make_config(5)           # 500k faces: many sort tiles, two rounds of subtrees
    print(f"static build: {big.faces.shape[1]} faces", flush=True)
    _pair(mg, big.verts0, big.faces, device)
    small = make_config(2)         # then a smaller tree on the scratch the first call left
    print(f"static build: {small.faces.shape[1]} faces", flush=True)
    _pair(mg, small.verts0, small.faces, device)
    rng = np.random.default_rng(7)
    P = rng.normal(size=(3, 4097)).astype(np.float32)   # points, a ragged tile
    print("static build: 4097 points", flush=True)
    _pair(mg, P, None, device)


def test_static_build_limits(device):
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd import _lib
    assert mg.lbvh_bytes(0, mg.MG_PRIM_POINTS) > 0
    # more primitives than the static scratch holds: rejected before any launch
    n = (1 << 20) + 1
    st = _lib.load().mg_lbvh_build_static(None, n, None, n, mg.MG_PRIM_POINTS, None, 0, None)
    assert st == 1                 # MG_ERR_INVALID_ARGUMENT
    # empty build
    e = _zeroed(mg, 0, mg.MG_PRIM_POINTS, device)
    mg.lbvh_build_static(torch.zeros((3, 0), dtype=torch.float32, device=device), None, e)
    torch.cuda.synchronize()
    assert int(host(e.buf[:256].view(torch.int32))[2]) == 0
