"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/lidar.h, the ctypes mirror matches the header, and the
pure-host calls behave (no GPU compute)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lidar.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lidar_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def A():
    from paper_2208_10295_amd import _abi
    return _abi


def test_every_declared_symbol_is_exported_and_bound(A):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(A.lib, n), f"{n} not exported by liblidar.so"
        assert n in A.SIGNATURES, f"{n} missing from the ctypes mirror"
    assert set(A.SIGNATURES) == set(names)


STRUCTS = {"SceneDesc": "lidar_scene_desc", "MaterialDesc": "lidar_material_desc", "SensorDesc": "lidar_sensor_desc",
           "Outputs": "lidar_outputs", "Params": "lidar_params", "Instance": "lidar_instance",
           "TuneDesc": "lidar_tune_desc", "TuneResult": "lidar_tune_result", "Stats": "lidar_stats",
           "SweepDesc": "lidar_sweep_desc", "SweepInfo": "lidar_sweep_info", "Actor": "lidar_actor",
           "EchoDesc": "lidar_echo_desc"}


def test_every_header_constant_is_mirrored(A):
    """Each numeric #define of the header (status codes, sentinels, scene flags, options) has the same value
    under the same name, without the LIDAR_ prefix, in the ctypes mirror."""
    txt = open(HEADER).read()
    found = re.findall(r"^#define LIDAR_([A-Z0-9_]+)\s+(-?(?:0x[0-9A-Fa-f]+|\d+))u?\b", txt, flags=re.M)
    assert len(found) >= 20
    for name, value in found:
        assert hasattr(A, name), name
        assert getattr(A, name) == int(value, 0), (name, value)


def test_struct_layouts_match_header(A, tmp_path):
    """Size and every field offset of the ctypes mirror equal what a C compiler sees in include/lidar.h."""
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lidar.h"', "int main(void) {"]
    for py, cname in STRUCTS.items():
        lines.append(f'printf("{py} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(A, py)._fields_:
            lines.append(f'printf("{py} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        struct, field, val = line.split()
        got[(struct, field)] = int(val)
    for py in STRUCTS:
        cls = getattr(A, py)
        assert got[(py, "size")] == C.sizeof(cls), py
        for fname, _ in cls._fields_:
            assert got[(py, fname)] == getattr(cls, fname).offset, (py, fname)


def test_scene_bytes_host_only(A):
    d = A.SceneDesc()
    d.n_vertices, d.n_triangles = 100, 50
    d.flags = A.SCENE_DEVICE_PTRS
    p, s = C.c_uint64(), C.c_uint64()
    assert A.lib.lidar_scene_bytes(C.byref(d), C.byref(p), C.byref(s)) == A.OK
    assert p.value >= 50 * (128 + 48 + 4) and p.value % 256 == 0
    d.flags = 0
    p2, s2 = C.c_uint64(), C.c_uint64()
    assert A.lib.lidar_scene_bytes(C.byref(d), C.byref(p2), C.byref(s2)) == A.OK
    assert s2.value >= s.value + 100 * 12 + 50 * 18       # room for the host-array copies
    d.n_triangles = 0
    assert A.lib.lidar_scene_bytes(C.byref(d), C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG
    d.n_triangles = 1 << 28
    assert A.lib.lidar_scene_bytes(C.byref(d), C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG
    assert A.lib.lidar_scene_bytes(None, C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG


def test_scene_size_limit_keeps_record_offsets_below_2gib(A):
    """The walk forms 32-bit byte offsets into buffers of at most 2^31 - 1 bytes: 44,739,242 triangles
    of 48 bytes fit (the last record ends 32 bytes below 2^31), one more is refused by the workspace
    queries of scenes and meshes (host-only, nothing is allocated)."""
    assert A.MAX_TRIANGLES == 44_739_242 and 48 * A.MAX_TRIANGLES <= 2 ** 31 - 1 < 48 * (A.MAX_TRIANGLES + 1)
    assert 128 * A.MAX_NODES <= 2 ** 31
    d = A.SceneDesc()
    d.n_vertices, d.flags = 3, A.SCENE_DEVICE_PTRS
    p, s = C.c_uint64(), C.c_uint64()
    for fn in (A.lib.lidar_scene_bytes, A.lib.lidar_mesh_bytes):
        d.n_triangles = 44_739_242
        assert fn(C.byref(d), C.byref(p), C.byref(s)) == A.OK
        assert p.value >= 48 * 44_739_242
        d.n_triangles = 44_739_243
        assert fn(C.byref(d), C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG


def test_origin_check_host_only(A):
    """The box padding 2^-20 M covers FP32 rounding for ray origins with every |p_i| <= M."""
    chk = A.lib.lidar_origin_check
    f3 = C.c_float * 3
    assert chk(100.0, f3(0.0, 0.0, 0.0)) == A.OK
    assert chk(100.0, f3(-100.0, 100.0, 99.9)) == A.OK                    # on the cube's faces
    assert chk(100.0, f3(0.0, 0.0, 100.01)) == A.WARN_ORIGIN_OUTSIDE_SCENE
    assert chk(100.0, f3(-3000.0, 0.0, 1.5)) == A.WARN_ORIGIN_OUTSIDE_SCENE
    assert chk(0.0, f3(0.0, 0.0, 0.0)) == A.OK
    assert chk(100.0, f3(float("nan"), 0.0, 0.0)) == A.ERR_INVALID_ARG
    assert chk(100.0, f3(float("inf"), 0.0, 0.0)) == A.ERR_INVALID_ARG
    assert chk(100.0, None) == A.ERR_INVALID_ARG
    assert A.WARN_ORIGIN_OUTSIDE_SCENE & A.WARN_WAVELENGTH_CLAMPED == 0   # warnings are bits


def test_null_context_calls_are_rejected(A):
    lib = A.lib
    assert lib.lidar_destroy(None) == A.OK
    assert lib.lidar_simulate(None, 0, 0, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_simulate_sweep(None, None, None, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_mesh_load(None, None, None, 0, None, 0, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_mesh_refit(None, 0, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_actors_set(None, None, 0, None, 0, None, 0, None) == A.ERR_INVALID_ARG
    assert lib.lidar_actors_update(None, None, 0, None) == A.ERR_INVALID_ARG
    assert lib.lidar_actors_clear(None) == A.ERR_INVALID_ARG
    assert lib.lidar_simulate_echoes(None, 0, 0, None, None, 0, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_echo_bytes(None, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_sensor_set(None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_materials_set(None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_backward(None, None, None, None, None, None, None, None, None, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_batch_destroy(None) == A.OK
    assert lib.lidar_batch_restarted(None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_set_option(None, A.OPT_BATCH_STACK, 0) == A.ERR_INVALID_ARG
    assert lib.lidar_tune(None, None, None, 0, None, 0, None, None, None, None, None) == A.ERR_INVALID_ARG
    assert lib.lidar_compact_points(None, None, 0, None, None, None, None, 0, None) == A.ERR_INVALID_ARG
    assert lib.lidar_create(0, None) == A.ERR_INVALID_ARG


def test_compact_workspace_sizes_host_only(A):
    w = C.c_uint64()
    for n, need in ((0, 256), (1, 256), (256 * 64, 256), (256 * 64 + 1, 512), (131072, 2048), (21385216, 334336)):
        assert A.lib.lidar_compact_bytes(n, C.byref(w)) == A.OK
        assert w.value == need and w.value >= 4 * ((n + 255) // 256), n
    assert A.lib.lidar_compact_bytes((1 << 31) + 1, C.byref(w)) == A.ERR_INVALID_ARG
    assert A.lib.lidar_compact_bytes(10, None) == A.ERR_INVALID_ARG


def test_create_without_gpu_reports_error(A):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = A.lib.lidar_create(0, C.byref(h))
    assert st in (A.ERR_HIP, A.ERR_INVALID_ARG)
    assert h.value is None
    assert len(A.lib.lidar_last_error(None)) > 0


def test_binding_fails_loudly_without_library(A, tmp_path):
    with pytest.raises(ImportError):
        A.load(str(tmp_path / "liblidar.so"))


def test_actor_workspace_sizes_host_only(A):
    p, s = C.c_uint64(), C.c_uint64()
    assert A.lib.lidar_actors_bytes(300, C.byref(p), C.byref(s)) == A.OK
    assert p.value >= 300 * (128 + 48 + 112 + 24) and p.value % 256 == 0 and s.value > 300 * 38
    assert A.lib.lidar_actors_bytes(0, C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG
    assert A.lib.lidar_actors_bytes((1 << 20) + 1, C.byref(p), C.byref(s)) == A.ERR_INVALID_ARG
    d = A.SceneDesc()
    d.n_vertices, d.n_triangles, d.flags = 100, 50, A.SCENE_DEVICE_PTRS
    assert A.lib.lidar_mesh_bytes(C.byref(d), C.byref(p), C.byref(s)) == A.OK
    assert p.value >= 50 * (128 + 48 + 4 + 12)


def test_probe_arguments_checked_on_the_host(A):
    """The bandwidth probes reject bad arguments before any launch (no GPU needed)."""
    P = C.c_void_p
    aligned, misaligned, sink = P(1 << 20), P((1 << 20) + 4), P(1 << 21)
    assert A.lib.lidar_probe_stream(None, 1 << 20, sink, None) == A.ERR_INVALID_ARG
    assert A.lib.lidar_probe_stream(aligned, 1 << 20, None, None) == A.ERR_INVALID_ARG
    assert A.lib.lidar_probe_stream(misaligned, 1 << 20, sink, None) == A.ERR_INVALID_ARG
    assert A.lib.lidar_probe_stream(aligned, 8, sink, None) == A.ERR_INVALID_ARG
    g = A.lib.lidar_probe_gather
    assert g(None, 1 << 20, 8, 4, 0, sink, None) == A.ERR_INVALID_ARG
    assert g(misaligned, 1 << 20, 8, 4, 1, sink, None) == A.ERR_INVALID_ARG
    assert g(aligned, 64, 8, 4, 0, sink, None) == A.ERR_INVALID_ARG             # less than one line
    assert g(aligned, (1 << 31) + 128, 8, 4, 0, sink, None) == A.ERR_INVALID_ARG  # beyond 32-bit offsets
    assert g(aligned, 1 << 20, 0, 4, 0, sink, None) == A.ERR_INVALID_ARG
    assert g(aligned, 1 << 20, 8, 0, 0, sink, None) == A.ERR_INVALID_ARG
    assert g(aligned, 1 << 20, 8, 4, 0, None, None) == A.ERR_INVALID_ARG
