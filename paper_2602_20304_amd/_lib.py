"""ctypes declarations of the C ABI in include/cm.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcm.so")

CM_OK = 0
STATUS = {0: "CM_OK", -1: "CM_ERR_INVALID_ARG", -2: "CM_ERR_OOM", -3: "CM_ERR_DEVICE", -4: "CM_ERR_NOT_READY",
          -5: "CM_ERR_REJECTED", -6: "CM_ERR_NOT_FOUND", -7: "CM_ERR_CAPACITY", -8: "CM_ERR_GEOMETRY"}
CM_MAX_K = 32
CM_NOALLOC_SCRATCH_BYTES = 64 << 20
TIMERS = {"broadphase": 0, "forward": 1, "backward": 2, "fused": 3, "ee_witness": 4}

vp = C.c_void_p
i32 = C.c_int32
i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)
f32p = C.POINTER(C.c_float)


class cm_params(C.Structure):
    _fields_ = [("tau", C.c_float), ("lambda_reg", C.c_float), ("eps_n", C.c_float), ("cull_margin", C.c_float),
                ("K", i32), ("flags", C.c_uint32), ("presel_vertices", i32), ("presel_edges", i32),
                ("refine_steps", i32)]


class cm_batch(C.Structure):
    _fields_ = [("n_scenes", i32), ("n_bodies", i32), ("body_offsets", vp), ("body_geom", vp), ("pose", vp),
                ("cand_offsets", vp), ("cand_pairs", vp), ("n_cand", i32)]


class cm_manifold(C.Structure):
    _fields_ = [("capacity", i32), ("n_pairs", vp), ("pair_offsets", vp), ("pairs", vp), ("point", vp),
                ("normal", vp), ("dist", vp), ("weight", vp), ("tape", vp), ("tape_bytes", C.c_int64)]


class cm_cotangent(C.Structure):
    _fields_ = [("g_point", vp), ("g_normal", vp), ("g_dist", vp), ("g_weight", vp)]


class cm_grads(C.Structure):
    _fields_ = [("g_pose", vp), ("g_vertices", vp), ("g_params", vp), ("g_tau", vp)]


class cm_geometry_info_t(C.Structure):
    _fields_ = [("type", i32), ("n_vertices", i32), ("n_edges", i32), ("n_faces", i32), ("vertex_offset", i32),
                ("bound_radius", C.c_float)]


class cm_request(C.Structure):
    _fields_ = [("n_scenes", i32), ("n_bodies", i32), ("body_offsets", vp), ("body_geom", vp), ("pose", vp),
                ("params", cm_params), ("want_backward", i32), ("cot_point", vp), ("cot_normal", vp),
                ("cot_dist", vp), ("cot_weight", vp), ("want_geometry_grads", i32), ("capacity", i32)]


class cm_result(C.Structure):
    _fields_ = [("status", i32), ("n_pairs", i32), ("capacity", i32), ("pair_offsets", i32p), ("pairs", i32p),
                ("point", f32p), ("normal", f32p), ("dist", f32p), ("weight", f32p), ("g_pose", f32p),
                ("g_tau", f32p), ("g_vertices", f32p), ("g_params", f32p), ("vertex_pool", i32),
                ("n_geometries", i32), ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("footprint_bytes", C.c_uint64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "cm_context_create": (i32, [C.c_int, C.POINTER(vp)]),
    "cm_context_destroy": (i32, [vp]),
    "cm_status_str": (C.c_char_p, [i32]),
    "cm_last_error": (C.c_char_p, [vp]),
    "cm_check_errors": (i32, [vp, vp]),
    "cm_geometry_create": (i32, [vp, i32, vp, vp, vp, vp, vp]),
    "cm_geometry_info": (i32, [vp, i32, C.POINTER(cm_geometry_info_t)]),
    "cm_geometry_mesh": (i32, [vp, i32, vp, vp, vp]),
    "cm_geometry_count": (i32, [vp]),
    "cm_vertex_pool_size": (i32, [vp]),
    "cm_geometry_destroy": (i32, [vp, vp, i32]),
    "cm_collide": (i32, [vp, C.POINTER(cm_batch), C.POINTER(cm_params), C.POINTER(cm_manifold), vp]),
    "cm_collide_fused": (i32, [vp, C.POINTER(cm_batch), C.POINTER(cm_params), C.POINTER(cm_manifold), vp]),
    "cm_fused_tuning": (i32, [vp, i32p, i32p, i32p, f32p, i32p]),
    "cm_collide_noalloc": (i32, [vp, C.POINTER(cm_batch), C.POINTER(cm_params), C.POINTER(cm_manifold), vp]),
    "cm_collide_backward": (i32, [vp, C.POINTER(cm_batch), C.POINTER(cm_params), C.POINTER(cm_manifold),
                                  C.POINTER(cm_cotangent), C.POINTER(cm_grads), vp]),
    "cm_ee_witness": (i32, [vp, vp, C.c_int64, C.c_float, C.c_float, i32, vp, vp]),
    "cm_tape_bytes": (i32, [vp, i32, i32, C.c_int64, C.POINTER(C.c_int64)]),
    "cm_set_kernel_timing": (i32, [vp, i32]),
    "cm_kernel_time": (i32, [vp, i32, C.POINTER(C.c_double), i64p]),
    "cm_server_create": (i32, [vp, C.c_uint64, i32, C.POINTER(vp)]),
    "cm_server_set_host_budget": (i32, [vp, C.c_uint64]),
    "cm_server_submit": (i32, [vp, C.POINTER(cm_request), C.POINTER(C.c_uint64)]),
    "cm_server_poll": (i32, [vp, C.c_uint64, C.POINTER(cm_result)]),
    "cm_server_release": (i32, [vp, C.c_uint64]),
    "cm_server_stats": (i32, [vp, C.POINTER(C.c_uint64), i32p, i32p]),
    "cm_server_destroy": (i32, [vp]),
    "cm_server_last_error": (C.c_char_p, []),
}

_lib = None


class CMError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libcm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2602_20304_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(SIGNATURES)
