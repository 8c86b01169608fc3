"""ctypes loader and prototypes for libmgu.so (the C ABI in include/mgu.h)."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgu.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U32 = ctypes.c_uint32
F32 = ctypes.c_float
SZ = ctypes.c_size_t

STATUS = {
    0: "MG_OK", 1: "MG_ERR_INVALID_ARGUMENT", 2: "MG_ERR_WORKSPACE_TOO_SMALL",
    3: "MG_ERR_INDEX_OUT_OF_RANGE", 4: "MG_ERR_NONFINITE_INPUT", 5: "MG_ERR_TOPOLOGY_MISMATCH",
    6: "MG_ERR_HIP", 7: "MG_ERR_UNSUPPORTED_DEVICE",
}
MG_PRIM_TRIANGLES = 0
MG_PRIM_POINTS = 1
MG_QUERY_AUTO = 0
MG_QUERY_LANE = 1
MG_QUERY_BATCH = 2


class MguError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {STATUS.get(code, code)}")
        self.code = code


class LbvhLayout(ctypes.Structure):
    _fields_ = [(n, I64) for n in ("total_bytes", "off_header", "off_codes", "off_prim", "off_leaf_faces",
                                   "off_leaf_parent", "off_node_parent", "off_nodes", "off_node_aux", "off_child",
                                   "off_top_nodes", "off_top_child", "off_subtrees",
                                   "off_deposits", "off_top_scratch", "off_inv_prim")]


class LbvhHeader(ctypes.Structure):
    _fields_ = [("n_prims", I32), ("prim_kind", I32), ("status", I32), ("n_verts", I32),
                ("root_lo", ctypes.c_float * 3), ("pad0", ctypes.c_float), ("root_hi", ctypes.c_float * 3),
                ("pad1", ctypes.c_float), ("quant_lo", ctypes.c_float * 3), ("quant_scale", ctypes.c_float * 3),
                ("bounds_enc", ctypes.c_uint32 * 6), ("tile_counter", ctypes.c_uint32 * 4), ("chunk_log2", I32),
                ("n_top", I32), ("n_sub", I32), ("refit_arrivals", ctypes.c_uint32),
                ("reserved", I32 * 8)]


class QueryOptions(ctypes.Structure):
    _fields_ = [("kernel", I32), ("batch", I32), ("seed", I32), ("warm", I32), ("order", P),
                ("counters", P), ("queue", P), ("hint", P), ("waves", I32)]


class BatchScene(ctypes.Structure):
    _fields_ = [("frames", P), ("n_frames", I32), ("n_verts", I32), ("faces", P), ("n_faces", I32),
                ("n_gauss", I32), ("gface", P), ("bary", P), ("q_local", P), ("log_scale", P),
                ("queries", P), ("n_queries", I32), ("batch", I32), ("seed", I32), ("query_tile", I32), ("bvh", P), ("bvh_bytes", SZ),
                ("nodes", P), ("roots", P), ("mean", P), ("quat", P), ("cov", P), ("face", P),
                ("point", P), ("qbary", P), ("dist2", P), ("normal", P)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("batch", I32), ("seed", I32), ("gauss_tile", I32), ("query_tile", I32), ("reserved", I32 * 4)]


# name -> (restype, argtypes); every symbol declared in include/mgu.h
PROTOTYPES = {
    "mg_status_string": (ctypes.c_char_p, [I32]),
    "mg_version": (I32, []),
    "mg_check_device": (I32, []),
    "mg_frame_index": (I32, [I64, I64, I64, I64, I32, P]),
    "mg_vertex_buffer_update": (I32, [P, I32, I32, I32, P, P]),
    "mg_fill": (I32, [P, I64, F32, P]),
    "mg_blend": (I32, [P, P, F32, F32, P, I64, P]),
    "mg_mesh_gaussian_update": (I32, [P, I32, P, I32, P, P, P, P, P, I32, U32, P, P, P, P, P]),
    "mg_mesh_gaussian_update_backward": (I32, [P, I32, P, I32, P, P, P, P, P, I32, P, P, P, P, P]),
    "mg_lbvh_layout_query": (I32, [I32, I32, P]),
    "mg_lbvh_workspace_size": (I32, [I32, I32, P]),
    "mg_lbvh_build": (I32, [P, I32, P, I32, I32, P, SZ, P, SZ, P]),
    "mg_lbvh_build_static": (I32, [P, I32, P, I32, I32, P, SZ, P]),
    "mg_frame_update": (I32, [P, I32, I32, I32, P, P, I32, P, P, P, P, P, I32, P, P, P, P, P, SZ, P]),
    "mg_lbvh_refit": (I32, [P, I32, P, SZ, I32, I32, P]),
    "mg_closest_point_query": (I32, [P, SZ, I32, P, I32, P, I32, F32, P, P, P, P, P, P, P]),
    "mg_closest_point_bruteforce": (I32, [P, I32, P, I32, P, I32, F32, P, P, P, P, P, P]),
    "mg_nearest_point_query": (I32, [P, SZ, I32, P, P, I32, F32, P, P, P, P]),
    "mg_particles_integrate": (I32, [P, P, I32, F32, F32, F32, F32, P]),
    "mg_contact_response": (I32, [P, P, I32, P, P, P, F32, F32, P, P]),
    "mg_grid_points": (I32, [F32, F32, F32, F32, I32, I32, I32, P, P]),
    "mg_sdf_update": (I32, [P, I32, P, I32, P, I32, F32, F32, F32, F32, I32, I32, I32, P, P, P]),
    "mg_sdf_sample": (I32, [P, F32, F32, F32, F32, I32, I32, I32, P, I32, P, P]),
    "mg_knn_surface_query": (I32, [P, SZ, I32, P, I32, P, I32, I32, F32, F32, P, P, P, P, P]),
    "mg_reduce_workspace_size": (I32, [I64, P]),
    "mg_mean": (I32, [P, I64, P, P, SZ, P]),
    "mg_chamfer": (I32, [P, I32, P, SZ, P, I32, P, SZ, P, P, P, P, P, P, P, SZ, P, P]),
    "mg_point_mesh_backward": (I32, [P, I32, P, I32, P, I32, P, P, P, F32, P, P, P]),
    "mg_chamfer_backward": (I32, [P, I32, P, I32, P, P, F32, F32, P, P, P]),
    "mg_adam_step": (I32, [P, P, P, P, I64, I32, F32, F32, F32, F32, P]),
    "mg_batch_plan_size": (I32, [P, I32, P]),
    "mg_batch_plan_init": (I32, [P, I32, P, P, SZ, P]),
    "mg_batch_run": (I32, [P, SZ, P]),
    "mg_batch_status_word": (I32, [P, P]),
    "mg_validate_indices": (I32, [P, I64, I32, P, P]),
    "mg_validate_finite": (I32, [P, I64, P, P]),
}

_lib = None


def load():
    """Load libmgu.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_00444_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(fn_name, code):
    if code != 0:
        raise MguError(fn_name, code)
