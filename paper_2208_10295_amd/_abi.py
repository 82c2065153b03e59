"""ctypes mirror of include/lidar.h (argument marshalling only).

Loads ``liblidar.so`` built in-tree by ``paper_2208_10295_amd/build.py``.  There
is no fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

# PyTorch ships its own HIP runtime; loading it before liblidar.so makes the
# library bind to that same runtime (one HIP runtime per process).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblidar.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_NOT_READY = -2
ERR_WORKSPACE_TOO_SMALL = -3
ERR_HIP = -4
ERR_UNSUPPORTED_DEVICE = -5
ERR_STACK_OVERFLOW = -6
ERR_NO_FORWARD_STATE = -7
ERR_OUT_OF_MEMORY = -8
WARN_WAVELENGTH_CLAMPED = 1
WARN_ORIGIN_OUTSIDE_SCENE = 2
MAX_TRIANGLES = 44739242
MAX_NODES = 16777216
MESH_REACH = 1024.0
COMPACT_NOALLOC_MAX_BEAMS = 33554432

NO_LABEL = 0xFFFFFFFF
NO_TRIANGLE = 0xFFFFFFFF
NO_MATERIAL = 0xFFFF
SCENE_DEVICE_PTRS = 1
SCENE_BUILD_LBVH = 2
SCENE_COLLAPSE_GREEDY = 4
OPT_TILE_AZ = 1
OPT_LANES_PER_RAY = 2
OPT_XCD_REMAP = 3
OPT_STACK_CAP = 4
OPT_ACTOR_TREE = 5
OPT_BATCH_STACK = 6

STATUS_NAMES = {
    OK: "OK", ERR_INVALID_ARG: "ERR_INVALID_ARG", ERR_NOT_READY: "ERR_NOT_READY",
    ERR_WORKSPACE_TOO_SMALL: "ERR_WORKSPACE_TOO_SMALL", ERR_HIP: "ERR_HIP",
    ERR_UNSUPPORTED_DEVICE: "ERR_UNSUPPORTED_DEVICE", ERR_STACK_OVERFLOW: "ERR_STACK_OVERFLOW",
    ERR_NO_FORWARD_STATE: "ERR_NO_FORWARD_STATE", ERR_OUT_OF_MEMORY: "ERR_OUT_OF_MEMORY",
    WARN_WAVELENGTH_CLAMPED: "WARN_WAVELENGTH_CLAMPED", WARN_ORIGIN_OUTSIDE_SCENE: "WARN_ORIGIN_OUTSIDE_SCENE",
}

P = C.c_void_p


class SceneDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_uint64), ("n_triangles", C.c_uint64), ("vertices", P), ("indices", P),
                ("material", P), ("label", P), ("leaf_width", C.c_uint32), ("flags", C.c_uint32)]


class MaterialDesc(C.Structure):
    _fields_ = [("nmat", C.c_uint32), ("nbins", C.c_uint32), ("lambda0_nm", C.c_float),
                ("dlambda_nm", C.c_float), ("spectra", P), ("sigma_range", P), ("angle_exp", P)]


class SensorDesc(C.Structure):
    _fields_ = [("n_ch", C.c_uint32), ("elev_deg", P), ("n_az", C.c_uint32), ("az0_deg", C.c_double),
                ("fov_h_deg", C.c_double), ("wavelength_nm", C.c_float), ("d_max", C.c_float),
                ("r_l_max", C.c_float), ("t_min", C.c_float), ("sigma_intensity", C.c_float),
                ("noise_on", C.c_uint32)]


class Outputs(C.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("intensity", P), ("label", P), ("valid", P), ("range", P),
                ("tri", P), ("t_hit", P), ("material", P), ("normal", P), ("r_lambda", P)]


class Params(C.Structure):
    _fields_ = [("rho", P), ("angle_exp", P), ("pose_delta", P), ("spectra", P)]


class Instance(C.Structure):
    _fields_ = [("sensor", SensorDesc), ("p", C.c_float * 3), ("q_wxyz", C.c_float * 4), ("seed", C.c_uint64),
                ("scan", C.c_uint32)]


class TuneDesc(C.Structure):
    _fields_ = [("packet_rays", P), ("n_packet", C.c_uint32), ("leaf_widths", P), ("n_leaf", C.c_uint32),
                ("lanes_per_ray", P), ("n_lanes", C.c_uint32), ("reps", C.c_uint32), ("up_weights", P),
                ("n_up", C.c_uint32)]


class TuneResult(C.Structure):
    _fields_ = [("best_packet_rays", C.c_uint32), ("best_leaf_width", C.c_uint32),
                ("best_lanes_per_ray", C.c_uint32), ("best_ms", C.c_float), ("ms", C.c_float * 64),
                ("best_up_weight", C.c_float)]


class Stats(C.Structure):
    _fields_ = [("n_triangles", C.c_uint64), ("n_nodes", C.c_uint64), ("n_leaves", C.c_uint64),
                ("depth", C.c_uint32), ("leaf_width", C.c_uint32), ("stack_entries", C.c_uint32),
                ("root", C.c_uint32), ("node_bytes", C.c_uint64), ("tri_bytes", C.c_uint64),
                ("build_ms", C.c_float), ("box_pad", C.c_float), ("max_abs_coord", C.c_float), ("pad_", C.c_uint32)]


class Actor(C.Structure):
    _fields_ = [("mesh", C.c_uint32), ("label", C.c_uint32), ("p", C.c_float * 3), ("q_wxyz", C.c_float * 4)]


class EchoDesc(C.Structure):
    _fields_ = [("n_sub", C.c_uint32), ("max_echoes", C.c_uint32), ("divergence_rad", C.c_float),
                ("echo_sep_m", C.c_float)]


class SweepDesc(C.Structure):
    _fields_ = [("head_deg", C.c_double), ("spin_hz", C.c_double), ("dt_s", C.c_double),
                ("p_begin", C.c_float * 3), ("q_begin", C.c_float * 4), ("p_end", C.c_float * 3),
                ("q_end", C.c_float * 4), ("seed", C.c_uint64)]


class SweepInfo(C.Structure):
    _fields_ = [("n_runs", C.c_uint32), ("n_columns", C.c_uint32), ("scan", C.c_uint32 * 2),
                ("first", C.c_uint32 * 2), ("count", C.c_uint32 * 2)]


# name -> (restype, argtypes); every entry point declared in include/lidar.h
SIGNATURES = {
    "lidar_create": (C.c_int32, [C.c_int, C.POINTER(P)]),
    "lidar_destroy": (C.c_int32, [P]),
    "lidar_last_error": (C.c_char_p, [P]),
    "lidar_scene_bytes": (C.c_int32, [C.POINTER(SceneDesc), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "lidar_scene_load": (C.c_int32, [P, C.POINTER(SceneDesc), P, C.c_uint64, P, C.c_uint64, P]),
    "lidar_materials_set": (C.c_int32, [P, C.POINTER(MaterialDesc)]),
    "lidar_sensor_set": (C.c_int32, [P, C.POINTER(SensorDesc)]),
    "lidar_pose_set": (C.c_int32, [P, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "lidar_origin_check": (C.c_int32, [C.c_float, C.POINTER(C.c_float)]),
    "lidar_set_option": (C.c_int32, [P, C.c_uint32, C.c_int32]),
    "lidar_simulate": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.POINTER(Outputs), P]),
    "lidar_simulate_ex": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.POINTER(Params), C.POINTER(Outputs), P]),
    "lidar_simulate_bruteforce": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.POINTER(Outputs), P]),
    "lidar_simulate_counts": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.POINTER(Outputs), P, P, P]),
    "lidar_compact_bytes": (C.c_int32, [C.c_uint64, C.POINTER(C.c_uint64)]),
    "lidar_compact_points": (C.c_int32, [P, C.POINTER(Outputs), C.c_uint64, C.POINTER(Outputs), P, P, P, C.c_uint64,
                                         P]),
    "lidar_compact_points_noalloc": (C.c_int32, [P, C.POINTER(Outputs), C.c_uint64, C.POINTER(Outputs), P, P, P]),
    "lidar_simulate_sweep": (C.c_int32, [P, C.POINTER(SweepDesc), C.POINTER(Outputs), C.POINTER(SweepInfo), P]),
    "lidar_probe_stream": (C.c_int32, [P, C.c_uint64, P, P]),
    "lidar_probe_gather": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, P, P]),
    "lidar_echo_bytes": (C.c_int32, [P, C.POINTER(EchoDesc), C.POINTER(C.c_uint64)]),
    "lidar_simulate_echoes": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.POINTER(EchoDesc), P, C.c_uint64,
                                          C.POINTER(Outputs), P]),
    "lidar_mesh_bytes": (C.c_int32, [C.POINTER(SceneDesc), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "lidar_mesh_load": (C.c_int32, [P, C.POINTER(SceneDesc), P, C.c_uint64, P, C.c_uint64, P,
                                    C.POINTER(C.c_uint32)]),
    "lidar_mesh_refit": (C.c_int32, [P, C.c_uint32, P, P]),
    "lidar_actors_bytes": (C.c_int32, [C.c_uint32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "lidar_actors_set": (C.c_int32, [P, C.POINTER(Actor), C.c_uint32, P, C.c_uint64, P, C.c_uint64, P]),
    "lidar_actors_update": (C.c_int32, [P, C.POINTER(Actor), C.c_uint32, P]),
    "lidar_actors_clear": (C.c_int32, [P]),
    "lidar_batch_create": (C.c_int32, [P, C.POINTER(Instance), C.c_uint32, C.c_uint32, C.POINTER(P)]),
    "lidar_batch_rays": (C.c_int32, [P, C.POINTER(C.c_uint64)]),
    "lidar_simulate_batch": (C.c_int32, [P, P, C.POINTER(Outputs), P]),
    "lidar_simulate_batch_sequential": (C.c_int32, [P, P, C.POINTER(Outputs), P]),
    "lidar_batch_restarted": (C.c_int32, [P, C.POINTER(C.c_uint64)]),
    "lidar_batch_destroy": (C.c_int32, [P]),
    "lidar_tune": (C.c_int32, [P, C.POINTER(SceneDesc), P, C.c_uint64, P, C.c_uint64, P, C.POINTER(Outputs),
                               C.POINTER(TuneDesc), C.POINTER(TuneResult), P]),
    "lidar_backward": (C.c_int32, [P, C.POINTER(Params), P, P, P, P, P, P, P, P, P]),
    "lidar_backward_spectra": (C.c_int32, [P, C.POINTER(Params), P, P, P, P, P, P, P, P, P]),
    "lidar_get_stats": (C.c_int32, [P, C.POINTER(Stats)]),
    "lidar_sync_check": (C.c_int32, [P, P]),
    "lidar_debug_copy_bvh": (C.c_int32, [P, P, C.c_uint64, P, C.c_uint64]),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2208_10295_amd/build.py` "
                          "(the LiDAR path has no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class LidarError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int, ctx=None) -> int:
    """Raise LidarError for errors; return the status (0 or a warning) otherwise."""
    if status < 0:
        msg = lib.lidar_last_error(ctx)
        raise LidarError(status, msg.decode() if msg else "")
    return status
