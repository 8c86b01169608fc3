"""The C-ABI library loads, exports every symbol declared in include/mgu.h, and rejects
bad arguments on the host before any HIP call (CPU only: no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mgu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_00444_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmgu.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2606_00444_amd import _lib
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mgu.h but not exported"
        assert n in _lib.PROTOTYPES, f"{n} has no ctypes prototype"


def test_host_only_calls(lib):
    assert lib.mg_version() == 100
    assert lib.mg_status_string(0) == b"MG_OK"
    assert lib.mg_status_string(5) == b"MG_ERR_TOPOLOGY_MISMATCH"
    k = ctypes.c_int32()
    assert lib.mg_frame_index(7, 30, 1, 30, 2, ctypes.byref(k)) == 0 and k.value == 1
    assert lib.mg_frame_index(59, 30, 1, 60, 100, ctypes.byref(k)) == 0 and k.value == 29
    assert lib.mg_frame_index(-1, 30, 1, 60, 100, ctypes.byref(k)) == 1
    assert lib.mg_frame_index(1, 30, 0, 60, 100, ctypes.byref(k)) == 1
    from paper_2606_00444_amd import _lib
    L = _lib.LbvhLayout()
    assert lib.mg_lbvh_layout_query(40000, 0, ctypes.byref(L)) == 0
    assert L.off_nodes % 256 == 0 and L.total_bytes >= 64 * 39999
    assert lib.mg_lbvh_layout_query(10, 7, ctypes.byref(L)) == 1
    ws = ctypes.c_size_t()
    assert lib.mg_lbvh_workspace_size(1_000_000, 0, ctypes.byref(ws)) == 0 and ws.value >= 16_000_000


def test_argument_errors_before_any_hip_call(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)   # never dereferenced: every case below fails validation first
    # negative / too large counts, null pointers, bad flags
    assert lib.mg_mesh_gaussian_update(fake, 10, fake, -1, fake, fake, fake, fake, None, 5, 0, fake, None, None,
                                       None, None) == 1
    assert lib.mg_mesh_gaussian_update(fake, 10, fake, 4, fake, fake, fake, fake, None, 5, 1, fake, None, None,
                                       None, None) == 1
    assert lib.mg_mesh_gaussian_update(None, 10, fake, 4, fake, fake, fake, fake, None, 5, 0, fake, None, None,
                                       None, None) == 1
    assert lib.mg_lbvh_build(fake, 3, fake, 1 << 30, 0, fake, 10, fake, 10, None) == 1
    assert lib.mg_lbvh_build(fake, 3, fake, 100, 0, fake, 10, fake, 10, None) == 2      # bvh too small
    assert lib.mg_lbvh_build(fake, 3, None, 4, 1, fake, 1 << 20, fake, 1 << 20, None) == 1   # points: n mismatch
    assert lib.mg_lbvh_refit(fake, 5, fake, 1 << 20, 7, 1, None) == 5                   # points, n mismatch
    assert lib.mg_closest_point_query(fake, 10, 100, fake, 3, fake, 5, ctypes.c_float(-1.0), fake, None, None,
                                      None, None, None, None) == 1
    assert lib.mg_closest_point_query(fake, 10, 100, fake, 3, fake, 5, ctypes.c_float(1.0), fake, None, None,
                                      None, None, None, None) == 2
    from paper_2606_00444_amd import _lib
    bad = _lib.QueryOptions()
    bad.kernel, bad.batch = 2, 3          # batch must be 0, 1, 2, 4, 8, 16 or 32
    assert lib.mg_closest_point_query(fake, 1 << 20, 100, fake, 3, fake, 5, ctypes.c_float(1.0), fake, None, None,
                                      None, None, ctypes.byref(bad), None) == 1
    bad.batch, bad.waves = 16, 3          # waves must be 0, 4 or 5
    assert lib.mg_closest_point_query(fake, 1 << 20, 100, fake, 3, fake, 5, ctypes.c_float(1.0), fake, None, None,
                                      None, None, ctypes.byref(bad), None) == 1
    from paper_2606_00444_amd import api
    with pytest.raises(ValueError):
        api._opts("batch", 16, waves=6)
    assert lib.mg_vertex_buffer_update(fake, 4, 10, 4, fake, None) == 1                 # k out of range
    assert lib.mg_adam_step(fake, fake, fake, fake, 10, 0, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                            ctypes.c_float(0.999), ctypes.c_float(1e-8), None) == 1
    assert lib.mg_mean(fake, 10, fake, None, 0, None) == 2


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the C structs' sizes and field offsets (gcc on the header)."""
    import subprocess
    from paper_2606_00444_amd import _lib
    structs = {"mg_lbvh_layout": _lib.LbvhLayout, "mg_lbvh_header": _lib.LbvhHeader,
               "mg_query_options": _lib.QueryOptions,
               "mg_batch_scene": _lib.BatchScene, "mg_batch_options": _lib.BatchOptions}
    lines = ['#include <stdio.h>', '#include "mgu.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_binding_rejects_vertex_counts_other_than_the_build(lib):
    """The kernels read vertices through the face ids stored at the build, unchecked, so
    the binding refuses a refit or query with another vertex count, and wrong dtypes,
    on the host (these raise before anything reaches the device)."""
    import torch
    import paper_2606_00444_amd as mg
    bvh = mg.LBVH(8, mg.MG_PRIM_TRIANGLES, "cpu")
    bvh.n_verts = 10
    q = torch.zeros(3, 4)
    with pytest.raises(ValueError, match="built on 10"):
        mg.lbvh_refit(bvh, torch.zeros(3, 9))
    with pytest.raises(ValueError, match="built on 10"):
        mg.closest_point_query(bvh, torch.zeros(3, 11), q)
    with pytest.raises(ValueError, match="built on 10"):
        mg.knn_surface_query(bvh, torch.zeros(3, 9), q)
    with pytest.raises(TypeError, match="float32"):
        mg.closest_point_query(bvh, torch.zeros(3, 10, dtype=torch.float64), q)
    with pytest.raises(ValueError, match=r"\[3\]\[n\]"):
        mg.lbvh_refit(bvh, torch.zeros(10, 3))
    pts = mg.LBVH(5, mg.MG_PRIM_POINTS, "cpu")
    with pytest.raises(ValueError, match="points has 6"):
        mg.nearest_point_query(pts, torch.zeros(3, 6), q)
