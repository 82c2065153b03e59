"""Python side of walk_replay.c: builds it with gcc and replays a scan's BVH walk on the CPU.

The replay walks the tree the GPU built (copied with lidar_debug_copy_bvh) with the
GPU walk's FP32 decisions and returns, per beam, the 4-wide nodes fetched and the
triangle records tested (the numerators of the trace kernel's algorithmic bytes),
plus its best hit, which must equal the GPU's.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "walk_replay.c")
LIB = os.path.join(HERE, "libwalk_replay.so")
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-std=c11", "-Wall", "-Wextra", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: run measure/walk_replay.py's build() (or __graft_entry__.build())")
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.walk_replay.restype = C.c_int64
        lib.walk_replay.argtypes = [P, P, C.c_uint32, P, C.c_uint32, C.c_uint32, C.c_double, C.c_double, P, P,
                                    C.c_float, C.c_float, P, C.c_int64, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def replay(nodes: np.ndarray, recs: np.ndarray, root: int, sensor, pose_p, pose_q, t_min: float, t_trace: float,
           beams=None, touched: bool = False, step_kinds: bool = False) -> dict:
    """Replays the walk for `beams` (default: every beam of the scan) of `sensor` (elev_deg, n_az, az0_deg,
    fov_h_deg) at pose (p, q).  nodes / recs: the device tree's bytes.  Returns dict of per-beam arrays:
    node_visits, tri_tests, leaf_visits (uint32), t (float32), orig (uint32), and the count of beams not
    replayed; with
    `touched`, also the numbers of distinct nodes and records the walks fetched."""
    lib = _load()
    n_ch = len(sensor.elev_deg)
    beams = np.arange(n_ch * int(sensor.n_az), dtype=np.uint32) if beams is None else \
        np.ascontiguousarray(beams, dtype=np.uint32)
    n = len(beams)
    nodes = np.ascontiguousarray(nodes).reshape(-1).view(np.uint8)     # the bytes, whatever the dtype
    recs = np.ascontiguousarray(recs).reshape(-1).view(np.uint8)
    elev = np.ascontiguousarray(sensor.elev_deg, dtype=np.float64)
    q = np.ascontiguousarray(pose_q, dtype=np.float32)
    p = np.ascontiguousarray(pose_p, dtype=np.float32)
    out = dict(node_visits=np.zeros(n, np.uint32), tri_tests=np.zeros(n, np.uint32),
               leaf_visits=np.zeros(n, np.uint32), t=np.zeros(n, np.float32), orig=np.zeros(n, np.uint32))
    nt_, nr_ = (nodes.size // 128, recs.size // 48) if touched else (0, 0)
    node_t, rec_t = np.zeros(nt_, np.uint8), np.zeros(nr_, np.uint8)
    kinds = np.zeros((n, 2), np.uint64) if step_kinds else None
    bad = lib.walk_replay(nodes.ctypes.data, recs.ctypes.data, int(root), elev.ctypes.data, n_ch, int(sensor.n_az),
                          float(sensor.az0_deg), float(sensor.fov_h_deg), q.ctypes.data, p.ctypes.data,
                          float(t_min), float(t_trace), beams.ctypes.data, n, out["node_visits"].ctypes.data,
                          out["tri_tests"].ctypes.data, out["leaf_visits"].ctypes.data, out["t"].ctypes.data,
                          out["orig"].ctypes.data,
                          node_t.ctypes.data if touched else None, rec_t.ctypes.data if touched else None,
                          kinds.ctypes.data if step_kinds else None)
    out["beams"] = beams
    out["not_replayed"] = int(bad)
    if step_kinds:
        out["leaf_steps"] = kinds          # bit i of word i // 64: step i is a leaf
    if touched:
        out["nodes_touched"] = int(node_t.sum(dtype=np.int64))
        out["records_touched"] = int(rec_t.sum(dtype=np.int64))
    return out


def trace_limit(sensor, sigma_range) -> float:
    """The scan's traceable range as the library forms it in FP32: d_max, plus 6.6605 x the largest
    range-noise sigma when the noise is on."""
    d = np.float32(sensor.d_max)
    if not sensor.noise_on:
        return float(d)
    return float(d + np.float32(6.6605) * np.float32(np.max(np.asarray(sigma_range, np.float32))))


if __name__ == "__main__":
    print(build())
