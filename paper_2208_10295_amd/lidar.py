"""Python binding of the gfx950 LiDAR library: argument marshalling only.

Every step of the simulation runs in the HIP kernels behind ``liblidar.so``;
this module converts arrays to the C structs of ``include/lidar.h``,
allocates outputs as PyTorch tensors (PyTorch supplies device memory and the
current stream) and raises ``LidarError`` on error statuses.
"""
from __future__ import annotations

import ctypes as C
import warnings

import numpy as np
import torch

from . import _abi as A
from ._abi import lib, check

POINT_OUTPUTS = ("x", "y", "z", "intensity", "label", "valid", "range")
DEBUG_OUTPUTS = ("tri", "t_hit", "material", "normal", "r_lambda")
_DTYPES = {"x": torch.float32, "y": torch.float32, "z": torch.float32, "intensity": torch.float32,
           "label": torch.int32, "valid": torch.uint8, "range": torch.float32, "tri": torch.int32,
           "t_hit": torch.float32, "material": torch.int16, "normal": torch.float32, "r_lambda": torch.float32}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _warn(status, what):
    """Turn the warning bits of a non-negative status into Python warnings; returns the status."""
    if status > 0 and status & A.WARN_WAVELENGTH_CLAMPED:
        warnings.warn(f"{what}: sensor wavelength outside the spectral table; end bin used", RuntimeWarning)
    if status > 0 and status & A.WARN_ORIGIN_OUTSIDE_SCENE:
        warnings.warn(f"{what}: a ray origin lies outside the cube the BVH's box padding covers; the walk may "
                      "rarely miss a hit the brute force finds", RuntimeWarning)
    return status


def as_u32(t: torch.Tensor) -> torch.Tensor:
    """View an int32 tensor holding u32 values as int64 with the unsigned values."""
    return t.to(torch.int64) & 0xFFFFFFFF


def alloc_outputs(n: int, names, device) -> dict:
    out = {}
    for k in names:
        shape = (3, n) if k == "normal" else (n,)
        out[k] = torch.empty(shape, dtype=_DTYPES[k], device=device)
    return out


def outputs_struct(out: dict) -> A.Outputs:
    s = A.Outputs()
    for k in ("x", "y", "z", "intensity", "label", "valid", "range", "tri", "t_hit", "material", "normal",
              "r_lambda"):
        t = out.get(k)
        if t is not None:
            assert t.is_cuda and t.is_contiguous()
            setattr(s, k, t.data_ptr())
    return s


def probe_stream_launcher(buf: torch.Tensor, sink: torch.Tensor, stream=None):
    """Callable that launches the HBM read probe over `buf` (lidar_probe_stream); one ctypes call each."""
    assert buf.is_cuda and buf.is_contiguous() and sink.is_cuda
    args = (C.c_void_p(buf.data_ptr()), C.c_uint64(buf.numel() * buf.element_size()), C.c_void_p(sink.data_ptr()),
            _stream(stream))
    fn = lib.lidar_probe_stream
    check(fn(*args))
    return lambda *_: fn(*args)


def probe_gather_launcher(table: torch.Tensor, blocks: int, steps: int, chase: bool, sink: torch.Tensor,
                          stream=None):
    """Callable that launches the 128-byte line gather probe over `table` (lidar_probe_gather)."""
    assert table.is_cuda and table.is_contiguous() and sink.is_cuda
    args = (C.c_void_p(table.data_ptr()), C.c_uint64(table.numel() * table.element_size()), C.c_uint32(blocks),
            C.c_uint32(steps), C.c_int32(1 if chase else 0), C.c_void_p(sink.data_ptr()), _stream(stream))
    fn = lib.lidar_probe_gather
    check(fn(*args))
    return lambda *_: fn(*args)


def sensor_struct(sensor):
    """lidar_sensor_desc from an object with the sensor attributes (keeps the elevation array alive)."""
    elev = np.ascontiguousarray(np.asarray(sensor.elev_deg, dtype=np.float64))
    d = A.SensorDesc()
    d.n_ch = len(elev)
    d.elev_deg = elev.ctypes.data
    d.n_az = int(sensor.n_az)
    d.az0_deg = float(getattr(sensor, "az0_deg", 0.0))
    d.fov_h_deg = float(getattr(sensor, "fov_h_deg", 360.0))
    d.wavelength_nm = float(sensor.wavelength_nm)
    d.d_max = float(sensor.d_max)
    d.r_l_max = float(getattr(sensor, "r_l_max", 0.8))
    d.t_min = float(getattr(sensor, "t_min", 0.01))
    d.sigma_intensity = float(getattr(sensor, "sigma_intensity", 0.0))
    d.noise_on = 1 if getattr(sensor, "noise_on", True) else 0
    return d, elev


class Context:
    """A library context on one HIP device (owns the scene workspace tensors)."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        check(lib.lidar_create(device, C.byref(h)), None)
        self.h = h
        self.persistent = None
        self.n_beams = 0
        self.scene_desc = None
        self._scene_keep = None
        self.nmat = 0

    def close(self):
        if getattr(self, "h", None):
            lib.lidar_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scene --------------------------------------------------------------
    def _scene_desc(self, vertices, indices, material, label, leaf_width, builder="ploc", ploc_radius=0,
                    collapse="sah", leaf_cost=0.0, up_weight=1.0):
        dev = self.device
        v = torch.as_tensor(np.ascontiguousarray(vertices, np.float32)).to(dev) if not torch.is_tensor(vertices) else vertices.to(dev, torch.float32).contiguous()
        i = torch.as_tensor(np.ascontiguousarray(indices, np.uint32).view(np.int32)).to(dev) if not torch.is_tensor(indices) else indices.to(dev, torch.int32).contiguous()
        m = torch.as_tensor(np.ascontiguousarray(material, np.uint16).view(np.int16)).to(dev) if not torch.is_tensor(material) else material.to(dev, torch.int16).contiguous()
        lab = torch.as_tensor(np.ascontiguousarray(label, np.uint32).view(np.int32)).to(dev) if not torch.is_tensor(label) else label.to(dev, torch.int32).contiguous()
        d = A.SceneDesc()
        d.n_vertices = v.shape[0]
        d.n_triangles = i.shape[0]
        d.vertices, d.indices, d.material, d.label = (t.data_ptr() for t in (v, i, m, lab))
        d.leaf_width = int(leaf_width)
        if builder not in ("ploc", "lbvh"):
            raise ValueError("builder must be 'ploc' or 'lbvh'")
        if collapse not in ("sah", "greedy"):
            raise ValueError("collapse must be 'sah' or 'greedy'")
        sixteenths = int(round(16 * leaf_cost))
        if not 0 <= sixteenths <= 255:
            raise ValueError("leaf_cost must be in [0, 255/16] (0 = default)")
        w128 = int(round(128 * up_weight))
        if not 1 <= w128 <= 255:
            raise ValueError("up_weight must be in [1/128, 255/128]")
        d.flags = (A.SCENE_DEVICE_PTRS | (A.SCENE_BUILD_LBVH if builder == "lbvh" else 0) | (int(ploc_radius) << 8) |
                   (A.SCENE_COLLAPSE_GREEDY if collapse == "greedy" else 0) | (sixteenths << 16) |
                   ((0 if w128 == 128 else w128) << 24))
        return d, (v, i, m, lab)

    def load_scene(self, vertices, indices, material, label, leaf_width: int = 4, stream=None, builder="ploc",
                   ploc_radius: int = 0, collapse: str = "sah", leaf_cost: float = 0.0, up_weight: float = 1.0):
        """Builds the scene BVH.  collapse: 'sah' (surface-area cost, leaf step weighing leaf_cost node
        steps, 0 = library default) or 'greedy'; up_weight: weight of a box's horizontal faces in the build's
        area metric (1 = surface area; below 1 for rays near the horizontal)."""
        d, keep = self._scene_desc(vertices, indices, material, label, leaf_width, builder, ploc_radius, collapse,
                                   leaf_cost, up_weight)
        pb, sb = C.c_uint64(), C.c_uint64()
        check(lib.lidar_scene_bytes(C.byref(d), C.byref(pb), C.byref(sb)), self.h)
        persistent = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        _warn(check(lib.lidar_scene_load(self.h, C.byref(d), _ptr(persistent), pb.value, _ptr(scratch), sb.value,
                                         _stream(stream)), self.h), "load_scene")
        del scratch
        self.persistent = persistent
        self.scene_desc = d
        self._scene_keep = keep
        return self.stats()

    def load(self, scene, leaf_width: int = 4, builder: str = "ploc", ploc_radius: int = 0, collapse: str = "sah",
             leaf_cost: float = 0.0, up_weight: float = 1.0):
        """Scene + materials from an object with vertices/indices/material/label/spectra/sigma_range/angle_exp."""
        st = self.load_scene(scene.vertices, scene.indices, scene.material, scene.label, leaf_width, builder=builder,
                             ploc_radius=ploc_radius, collapse=collapse, leaf_cost=leaf_cost, up_weight=up_weight)
        self.set_materials(scene.spectra, scene.sigma_range, scene.angle_exp)
        return st

    # -- dynamic scenes -----------------------------------------------------
    def load_mesh(self, mesh, leaf_width: int = 4, stream=None) -> int:
        """Builds the BVH of a mesh (object-space vertices/indices/material); returns its id."""
        dev = self.device
        v = torch.as_tensor(np.ascontiguousarray(mesh.vertices, np.float32)).to(dev)
        i = torch.as_tensor(np.ascontiguousarray(mesh.indices, np.uint32).view(np.int32)).to(dev)
        m = torch.as_tensor(np.ascontiguousarray(mesh.material, np.uint16).view(np.int16)).to(dev)
        d = A.SceneDesc()
        d.n_vertices, d.n_triangles = v.shape[0], i.shape[0]
        d.vertices, d.indices, d.material = v.data_ptr(), i.data_ptr(), m.data_ptr()
        d.leaf_width = int(leaf_width)
        d.flags = A.SCENE_DEVICE_PTRS
        pb, sb = C.c_uint64(), C.c_uint64()
        check(lib.lidar_mesh_bytes(C.byref(d), C.byref(pb), C.byref(sb)), self.h)
        persistent = torch.empty(pb.value, dtype=torch.uint8, device=dev)
        scratch = torch.empty(sb.value, dtype=torch.uint8, device=dev)
        mid = C.c_uint32()
        check(lib.lidar_mesh_load(self.h, C.byref(d), _ptr(persistent), pb.value, _ptr(scratch), sb.value,
                                  _stream(stream), C.byref(mid)), self.h)
        if not hasattr(self, "_meshes"):
            self._meshes = []
        self._meshes.append((persistent, int(v.shape[0])))
        return int(mid.value)

    def refit_mesh(self, mesh_id: int, vertices, stream=None):
        """New object-space vertices for a loaded mesh (same topology); call update_actors afterwards."""
        t = vertices if torch.is_tensor(vertices) else torch.as_tensor(np.ascontiguousarray(vertices, np.float32))
        t = t.to(self.device, torch.float32).contiguous()
        assert t.shape == (self._meshes[mesh_id][1], 3)
        check(lib.lidar_mesh_refit(self.h, int(mesh_id), _ptr(t), _stream(stream)), self.h)
        self._refit_keep = t      # alive until the stream has used it

    @staticmethod
    def _actor_array(actors):
        arr = (A.Actor * len(actors))()
        for k, a in enumerate(actors):
            arr[k].mesh, arr[k].label = int(a.mesh), int(a.label)
            for e in range(3):
                arr[k].p[e] = float(a.p[e])
            for e in range(4):
                arr[k].q_wxyz[e] = float(a.q[e])
        return arr

    def set_actors(self, actors, stream=None):
        """Places meshes by actors (objects with mesh, label, p, q) and builds the top-level BVH."""
        n = len(actors)
        if n == 0:
            self.clear_actors()
            return
        pb, sb = C.c_uint64(), C.c_uint64()
        check(lib.lidar_actors_bytes(n, C.byref(pb), C.byref(sb)), self.h)
        persistent = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        arr = self._actor_array(actors)
        check(lib.lidar_actors_set(self.h, arr, n, _ptr(persistent), pb.value, _ptr(scratch), sb.value,
                                   _stream(stream)), self.h)
        self._actors_persistent = persistent

    def update_actors(self, actors, stream=None):
        """Same actors at new poses: top-level BVH refit (asynchronous).  `actors` may be a
        prebuilt array from actor_array()."""
        arr = actors if isinstance(actors, C.Array) else self._actor_array(actors)
        check(lib.lidar_actors_update(self.h, arr, len(arr), _stream(stream)), self.h)

    actor_array = _actor_array

    def clear_actors(self):
        check(lib.lidar_actors_clear(self.h), self.h)
        self._actors_persistent = None

    def stats(self) -> dict:
        s = A.Stats()
        check(lib.lidar_get_stats(self.h, C.byref(s)), self.h)
        return {k: getattr(s, k) for k, _ in A.Stats._fields_}

    # -- materials / sensor / pose -----------------------------------------
    def set_materials(self, spectra, sigma_range, angle_exp=None, lambda0_nm: float = 400.0,
                      dlambda_nm: float = 10.0):
        sp = np.ascontiguousarray(spectra, np.float32)
        sg = np.ascontiguousarray(sigma_range, np.float32)
        ke = None if angle_exp is None else np.ascontiguousarray(angle_exp, np.float32)
        d = A.MaterialDesc()
        d.nmat, d.nbins = sp.shape
        d.lambda0_nm, d.dlambda_nm = lambda0_nm, dlambda_nm
        d.spectra = sp.ctypes.data
        d.sigma_range = sg.ctypes.data
        d.angle_exp = None if ke is None else ke.ctypes.data
        check(lib.lidar_materials_set(self.h, C.byref(d)), self.h)
        self.nmat = int(d.nmat)
        self.nbins = int(d.nbins)

    def set_sensor(self, sensor) -> int:
        d, keep = sensor_struct(sensor)
        st = check(lib.lidar_sensor_set(self.h, C.byref(d)), self.h)
        self.n_beams = int(d.n_ch) * int(d.n_az)
        return _warn(st, "set_sensor")

    def set_pose(self, p, q):
        pa = (C.c_float * 3)(*[float(x) for x in p])
        qa = (C.c_float * 4)(*[float(x) for x in q])
        return _warn(check(lib.lidar_pose_set(self.h, pa, qa), self.h), "set_pose")

    def set_tile_shape(self, tile_az: int):
        check(lib.lidar_set_option(self.h, A.OPT_TILE_AZ, int(tile_az)), self.h)

    def set_lanes_per_ray(self, lanes: int):
        check(lib.lidar_set_option(self.h, A.OPT_LANES_PER_RAY, int(lanes)), self.h)

    def set_xcd_remap(self, on: bool):
        check(lib.lidar_set_option(self.h, A.OPT_XCD_REMAP, 1 if on else 0), self.h)

    def set_actor_tree(self, mode: int):
        """0: top-level tree rebuilt by every update (up to 4,096 actors); 1: builder's tree, refit by updates.
        Read by the next set_actors."""
        check(lib.lidar_set_option(self.h, A.OPT_ACTOR_TREE, int(mode)), self.h)

    def set_batch_stack(self, entries: int):
        """First-pass stack of batched launches: 0 automatic, -1 off, n > 0 at most n entries (rays that need
        more are traced again with the whole stack; results never change)."""
        check(lib.lidar_set_option(self.h, A.OPT_BATCH_STACK, int(entries)), self.h)

    def batch_restarted(self) -> int:
        """Rays the last batched launch traced again with the whole stack (waits for the device)."""
        n = C.c_uint64()
        check(lib.lidar_batch_restarted(self.h, C.byref(n)), self.h)
        return int(n.value)

    def set_stack_cap(self, entries: int):
        """Limit the traversal stack of static-scene walks to `entries` (0 = no limit).  Only for testing
        the overflow path: results of walks that overflow are wrong and sync_check() raises."""
        check(lib.lidar_set_option(self.h, A.OPT_STACK_CAP, int(entries)), self.h)

    # -- simulation ---------------------------------------------------------
    def simulate(self, seed: int = 0, scan: int = 0, debug: bool = False, out: dict | None = None,
                 params: dict | None = None, stream=None, bruteforce: bool = False) -> dict:
        if out is None:
            out = alloc_outputs(self.n_beams, POINT_OUTPUTS + (DEBUG_OUTPUTS if debug else ()), self.device)
        o = outputs_struct(out)
        if bruteforce:
            st = lib.lidar_simulate_bruteforce(self.h, seed, scan, C.byref(o), _stream(stream))
        elif params:
            p = A.Params()
            for k in ("rho", "angle_exp", "pose_delta", "spectra"):
                t = params.get(k)
                if t is not None:
                    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                    setattr(p, k, t.data_ptr())
            st = lib.lidar_simulate_ex(self.h, seed, scan, C.byref(p), C.byref(o), _stream(stream))
        else:
            st = lib.lidar_simulate(self.h, seed, scan, C.byref(o), _stream(stream))
        check(st, self.h)
        return out

    def scan_launcher(self, seed: int, out: dict, params: dict | None = None, stream=None):
        """A callable f(scan) that runs lidar_simulate (lidar_simulate_ex with `params`) on fixed
        outputs and stream.

        The argument structs are built once, so a loop of f(k) costs one ctypes
        call per scan on the host (for back-to-back launches that keep the GPU
        queue full)."""
        o = outputs_struct(out)
        ob = C.byref(o)
        sp = _stream(stream)
        h = self.h
        seed = int(seed)
        if params:
            p = _params_struct(params)
            pb = C.byref(p)
            fn = lib.lidar_simulate_ex

            def run(scan: int):
                st = fn(h, seed, scan, pb, ob, sp)
                if st < 0:
                    check(st, h)
            run._keep = (o, out, p, params)
            return run
        fn = lib.lidar_simulate

        def run(scan: int):
            st = fn(h, seed, scan, ob, sp)
            if st < 0:
                check(st, h)
        run._keep = (o, out)
        return run

    def trajectory_launcher(self, seed: int, out: dict, poses, stream=None):
        """A callable f(k) that sets pose k of `poses` (objects with p and q) and runs scan k on fixed
        outputs and stream: a trajectory replayed one scan per tick.  The pose arrays and argument structs
        are built once, so f(k) costs two ctypes calls on the host."""
        o = outputs_struct(out)
        ob = C.byref(o)
        sp = _stream(stream)
        h = self.h
        seed = int(seed)
        pa = [(C.c_float * 3)(*[float(x) for x in ps.p]) for ps in poses]
        qa = [(C.c_float * 4)(*[float(x) for x in ps.q]) for ps in poses]
        set_pose, sim = lib.lidar_pose_set, lib.lidar_simulate

        def run(k: int):
            st = set_pose(h, pa[k], qa[k])
            if st < 0:
                check(st, h)
            st = sim(h, seed, k, ob, sp)
            if st < 0:
                check(st, h)
        run._keep = (o, out, pa, qa)
        return run

    def backward_launcher(self, tri, valid, dL_dI, dL_drange, params: dict | None = None, spectra: bool = False,
                          stream=None, intensity=None):
        """A callable f() that runs lidar_backward (lidar_backward_spectra if `spectra`) with fixed
        arguments, writing into the returned (d_rho or d_spectra, d_k, d_pose6) tensors."""
        nmat = self.nmat
        shape = (nmat, self.nbins) if spectra else (nmat,)
        d_a = torch.empty(shape, dtype=torch.float32, device=self.device)
        d_k = torch.empty(nmat, dtype=torch.float32, device=self.device)
        d_pose = torch.empty(6, dtype=torch.float32, device=self.device)
        p = _params_struct(params)
        args = (self.h, C.byref(p), _ptr(tri), _ptr(valid), _ptr(intensity), _ptr(dL_dI), _ptr(dL_drange), _ptr(d_a),
                _ptr(d_k), _ptr(d_pose), _stream(stream))
        fn = lib.lidar_backward_spectra if spectra else lib.lidar_backward
        h = self.h

        def run(*_):
            st = fn(*args)
            if st < 0:
                check(st, h)
        run._keep = (p, params, tri, valid, intensity, dL_dI, dL_drange)
        return run, (d_a, d_k, d_pose)

    def compact(self, dense: dict, names=None, out: dict | None = None, workspace=None, stream=None,
                read_count: bool = True, noalloc: bool = False):
        """Order-preserving compaction of dense outputs (any number of beams) to the detected points.

        Returns (points, beam_index, count): `points` maps each requested name (default: every dense
        array) to a tensor of capacity n whose first `count` elements are the detected points in beam
        order, `beam_index` their dense indices, `count` the device count tensor, or its value (a host
        int, after a synchronisation) if read_count is True; then the tensors are cut to that length.
        noalloc: use lidar_compact_points_noalloc (the library's static scratch, no workspace)."""
        v = dense.get("valid")
        n = int(v.numel()) if v is not None else int(next(t for t in dense.values() if t is not None).shape[-1])
        dense = {k: t for k, t in dense.items() if t is not None}
        names = tuple(dense.keys()) if names is None else tuple(names)
        if out is None:
            out = alloc_outputs(n, names, self.device)
        beam_index = torch.empty(n, dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int32, device=self.device)
        di, co = outputs_struct(dense), outputs_struct({k: out[k] for k in names})
        if noalloc:
            check(lib.lidar_compact_points_noalloc(self.h, C.byref(di), n, C.byref(co), _ptr(beam_index),
                                                   _ptr(count), _stream(stream)), self.h)
        else:
            nbytes = C.c_uint64()
            check(lib.lidar_compact_bytes(n, C.byref(nbytes)), self.h)
            if workspace is None or workspace.numel() < nbytes.value:
                workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            check(lib.lidar_compact_points(self.h, C.byref(di), n, C.byref(co), _ptr(beam_index), _ptr(count),
                                           _ptr(workspace), workspace.numel(), _stream(stream)), self.h)
            self._compact_workspace = workspace
        if not read_count:
            return out, beam_index, count
        c = int(count.item())
        pts = {k: (v[:, :c] if k == "normal" else v[:c]) for k, v in out.items()}
        return pts, beam_index[:c], c

    def compact_launcher(self, dense: dict, out: dict, stream=None):
        """A callable f() that runs lidar_compact_points on fixed arrays; returns (f, beam_index, count)
        with count a one-element device tensor."""
        n = int(dense["valid"].numel())
        nbytes = C.c_uint64()
        check(lib.lidar_compact_bytes(n, C.byref(nbytes)), self.h)
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        beam_index = torch.empty(n, dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int32, device=self.device)
        di, co = outputs_struct(dense), outputs_struct(out)
        args = (self.h, C.byref(di), n, C.byref(co), _ptr(beam_index), _ptr(count), _ptr(ws), ws.numel(),
                _stream(stream))
        fn, h = lib.lidar_compact_points, self.h

        def run(*_):
            st = fn(*args)
            if st < 0:
                check(st, h)
        run._keep = (di, co, ws, dense, out)
        return run, beam_index, count

    def simulate_sweep(self, seed: int, head_deg: float, spin_hz: float, dt_s: float, pose_begin, pose_end,
                       out: dict | None = None, debug: bool = False, stream=None):
        """One engine tick: traces the columns the head fires over
        [head_deg, head_deg + 360 spin_hz dt_s) with rolling-shutter poses
        interpolated from pose_begin = (p, q) to pose_end = (p, q).  Writes the
        fired columns' beams into the [n_ch][n_az] outputs `out` (allocated and
        zero-filled if None) and returns (out, info) with info = the fired runs
        [(scan, first_azimuth, count), ...]."""
        if out is None:
            out = alloc_outputs(self.n_beams, POINT_OUTPUTS + (DEBUG_OUTPUTS if debug else ()), self.device)
            for t in out.values():
                t.zero_()
        d = A.SweepDesc()
        d.head_deg, d.spin_hz, d.dt_s, d.seed = float(head_deg), float(spin_hz), float(dt_s), int(seed)
        for name, val in (("p_begin", pose_begin[0]), ("q_begin", pose_begin[1]), ("p_end", pose_end[0]),
                          ("q_end", pose_end[1])):
            arr = getattr(d, name)
            for k, x in enumerate(np.asarray(val, dtype=np.float32).reshape(-1)):
                arr[k] = float(x)
        info = A.SweepInfo()
        o = outputs_struct(out)
        _warn(check(lib.lidar_simulate_sweep(self.h, C.byref(d), C.byref(o), C.byref(info), _stream(stream)), self.h),
              "simulate_sweep")
        runs = [(int(info.scan[r]), int(info.first[r]), int(info.count[r])) for r in range(info.n_runs)]
        return out, runs

    def simulate_echoes(self, seed: int, scan: int, n_sub: int, max_echoes: int, divergence_rad: float,
                        echo_sep_m: float, debug: bool = False, out: dict | None = None, workspace=None,
                        stream=None):
        """One scan with divergent beams (n_sub sub-rays in a cone of full angle divergence_rad) and
        up to max_echoes echoes per beam.  Returns a dict of [max_echoes, n_beams] tensors."""
        d = A.EchoDesc(int(n_sub), int(max_echoes), float(divergence_rad), float(echo_sep_m))
        nbytes = C.c_uint64()
        check(lib.lidar_echo_bytes(self.h, C.byref(d), C.byref(nbytes)), self.h)
        if workspace is None or workspace.numel() < nbytes.value:
            workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        names = POINT_OUTPUTS + (tuple(k for k in DEBUG_OUTPUTS if k != "normal") if debug else ())
        if out is None:
            out = alloc_outputs(self.n_beams * int(max_echoes), names, self.device)
        o = outputs_struct(out)
        st = lib.lidar_simulate_echoes(self.h, int(seed), int(scan), C.byref(d), _ptr(workspace), workspace.numel(),
                                       C.byref(o), _stream(stream))
        check(st, self.h)
        self._echo_workspace = workspace
        return {k: v.view(int(max_echoes), self.n_beams) for k, v in out.items()}

    def simulate_counts(self, seed: int = 0, scan: int = 0, stream=None):
        """One scan plus per-beam (node visits, triangle tests) of the traversal."""
        out = alloc_outputs(self.n_beams, POINT_OUTPUTS, self.device)
        nn = torch.empty(self.n_beams, dtype=torch.int32, device=self.device)
        nt = torch.empty(self.n_beams, dtype=torch.int32, device=self.device)
        o = outputs_struct(out)
        check(lib.lidar_simulate_counts(self.h, seed, scan, C.byref(o), _ptr(nn), _ptr(nt), _stream(stream)),
              self.h)
        return out, nn, nt

    def sync_check(self, stream=None):
        check(lib.lidar_sync_check(self.h, _stream(stream)), self.h)

    def backward(self, tri, valid, dL_dI=None, dL_drange=None, params: dict | None = None, stream=None,
                 intensity=None):
        """Adjoint of one scan: (d_rho, d_k, d_pose6).  `intensity` is the forward's intensity output,
        required when the sensor has intensity noise (its clamp at 0 stops the gradient)."""
        nmat = self.nmat
        d_rho = torch.empty(nmat, dtype=torch.float32, device=self.device)
        d_k = torch.empty(nmat, dtype=torch.float32, device=self.device)
        d_pose = torch.empty(6, dtype=torch.float32, device=self.device)
        p = _params_struct(params)
        check(lib.lidar_backward(self.h, C.byref(p), _ptr(tri), _ptr(valid), _ptr(intensity), _ptr(dL_dI),
                                 _ptr(dL_drange), _ptr(d_rho), _ptr(d_k), _ptr(d_pose), _stream(stream)), self.h)
        return d_rho, d_k, d_pose

    def backward_spectra(self, tri, valid, dL_dI=None, dL_drange=None, params: dict | None = None, stream=None,
                         intensity=None):
        """Full-spectrum adjoint: (d_spectra[nmat, nbins], d_k[nmat], d_pose6) at the sensor wavelength."""
        d_T = torch.empty((self.nmat, self.nbins), dtype=torch.float32, device=self.device)
        d_k = torch.empty(self.nmat, dtype=torch.float32, device=self.device)
        d_pose = torch.empty(6, dtype=torch.float32, device=self.device)
        p = _params_struct(params)
        check(lib.lidar_backward_spectra(self.h, C.byref(p), _ptr(tri), _ptr(valid), _ptr(intensity), _ptr(dL_dI),
                                         _ptr(dL_drange), _ptr(d_T), _ptr(d_k), _ptr(d_pose), _stream(stream)),
              self.h)
        return d_T, d_k, d_pose

    def batch(self, instances, packet_rays: int = 0) -> "Batch":
        return Batch(self, instances, packet_rays)

    def debug_bvh(self):
        s = self.stats()
        nodes = np.empty(s["n_nodes"] * 128, np.uint8)
        tris = np.empty(s["n_triangles"] * 48, np.uint8)
        check(lib.lidar_debug_copy_bvh(self.h, nodes.ctypes.data, nodes.nbytes, tris.ctypes.data, tris.nbytes),
              self.h)
        return nodes, tris


class Batch:
    """Many sensor instances simulated by one persistent, graph-captured launch."""

    def __init__(self, ctx: Context, instances, packet_rays: int = 0):
        self.ctx = ctx
        arr = (A.Instance * len(instances))()
        keep = []
        for k, inst in enumerate(instances):
            d, elev = sensor_struct(inst.sensor)
            keep.append(elev)
            arr[k].sensor = d
            arr[k].p[:] = [float(x) for x in inst.pose.p]
            arr[k].q_wxyz[:] = [float(x) for x in inst.pose.q]
            arr[k].seed = int(inst.seed)
            arr[k].scan = int(inst.scan)
        h = C.c_void_p()
        st = check(lib.lidar_batch_create(ctx.h, arr, len(instances), int(packet_rays), C.byref(h)), ctx.h)
        self.clamped = bool(st & A.WARN_WAVELENGTH_CLAMPED)
        self.origin_outside = bool(st & A.WARN_ORIGIN_OUTSIDE_SCENE)
        self.h = h
        n = C.c_uint64()
        check(lib.lidar_batch_rays(h, C.byref(n)), ctx.h)
        self.n_rays = int(n.value)
        offs = np.zeros(len(instances) + 1, np.int64)
        offs[1:] = np.cumsum([len(i.sensor.elev_deg) * int(i.sensor.n_az) for i in instances])
        self.offsets = offs

    def simulate(self, out: dict | None = None, debug: bool = False, stream=None, sequential: bool = False):
        if out is None:
            out = alloc_outputs(self.n_rays, POINT_OUTPUTS + (DEBUG_OUTPUTS if debug else ()), self.ctx.device)
        o = outputs_struct(out)
        fn = lib.lidar_simulate_batch_sequential if sequential else lib.lidar_simulate_batch
        check(fn(self.ctx.h, self.h, C.byref(o), _stream(stream)), self.ctx.h)
        return out

    def tune(self, packet_rays=(64, 128, 256, 512), leaf_widths=(2, 4, 8), lanes_per_ray=(1, 4), reps=5, out=None,
             stream=None, up_weights=None):
        """Autotunes the batch (lidar_tune).  up_weights: candidate weights of the horizontal faces in the tree
        build's area metric (None: the scene's own); with them the timing grid has a leading weight axis."""
        ctx = self.ctx
        if out is None:
            out = alloc_outputs(self.n_rays, POINT_OUTPUTS, ctx.device)
        o = outputs_struct(out)
        pk = np.ascontiguousarray(packet_rays, np.uint32)
        lw = np.ascontiguousarray(leaf_widths, np.uint32)
        ln = np.ascontiguousarray(lanes_per_ray, np.uint32)
        uw = None if up_weights is None else np.ascontiguousarray(up_weights, np.float32)
        d = A.TuneDesc(pk.ctypes.data, len(pk), lw.ctypes.data, len(lw), ln.ctypes.data, len(ln), int(reps),
                       None if uw is None else uw.ctypes.data, 0 if uw is None else len(uw))
        r = A.TuneResult()
        sd = ctx.scene_desc
        pb, sb = C.c_uint64(), C.c_uint64()
        check(lib.lidar_scene_bytes(C.byref(sd), C.byref(pb), C.byref(sb)), ctx.h)
        scratch = torch.empty(sb.value, dtype=torch.uint8, device=ctx.device)
        check(lib.lidar_tune(ctx.h, C.byref(sd), _ptr(ctx.persistent), ctx.persistent.numel(), _ptr(scratch),
                             sb.value, self.h, C.byref(o), C.byref(d), C.byref(r), _stream(stream)), ctx.h)
        nu = 1 if uw is None else len(uw)
        grid = np.array(r.ms[:nu * len(pk) * len(lw) * len(ln)], np.float64).reshape(nu, len(lw), len(ln), len(pk))
        if uw is None:
            grid = grid[0]
        return dict(best_packet_rays=r.best_packet_rays, best_leaf_width=r.best_leaf_width,
                    best_lanes_per_ray=r.best_lanes_per_ray, best_ms=r.best_ms, best_up_weight=r.best_up_weight,
                    ms=grid, packet_rays=list(pk), leaf_widths=list(lw), lanes_per_ray=list(ln),
                    up_weights=None if uw is None else [float(x) for x in uw])

    def close(self):
        if getattr(self, "h", None):
            lib.lidar_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params_struct(params: dict | None) -> A.Params:
    p = A.Params()
    for k in ("rho", "angle_exp", "pose_delta", "spectra"):
        t = (params or {}).get(k)
        if t is not None:
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            setattr(p, k, t.data_ptr())
    return p


class LidarReturn(torch.autograd.Function):
    """(rho[nmat], k[nmat], pose_delta[6]) -> (intensity, range, valid, tri) of one scan.

    The backward pass is the library's adjoint kernel with the hit triangles
    of the forward pass held fixed; the pose gradient is with respect to
    pose_delta = (dp, dw) with p = p0 + dp and R = Exp(dw) R0.  With the
    sensor's noise on, the range noise is additive (its gradient is the
    range's) and the intensity clamp max(0, R_lambda + sigma_I z) stops the
    gradient where it holds (the forward's intensity is saved for that).
    """

    @staticmethod
    def forward(ctx_, lidar_ctx: Context, rho, k, pose_delta, seed: int = 0, scan: int = 0):
        out = lidar_ctx.simulate(seed, scan, out=alloc_outputs(lidar_ctx.n_beams, ("intensity", "range", "valid",
                                                                                  "tri"), lidar_ctx.device),
                                 params=dict(rho=rho.detach().contiguous(), angle_exp=k.detach().contiguous(),
                                             pose_delta=pose_delta.detach().contiguous()))
        ctx_.lidar = lidar_ctx
        ctx_.save_for_backward(rho, k, pose_delta, out["tri"], out["valid"], out["intensity"])
        ctx_.mark_non_differentiable(out["valid"], out["tri"])
        return out["intensity"], out["range"], out["valid"], out["tri"]

    @staticmethod
    def backward(ctx_, gI, gR, _gv, _gt):
        rho, k, pose_delta, tri, valid, inten = ctx_.saved_tensors
        d_rho, d_k, d_pose = ctx_.lidar.backward(
            tri, valid, None if gI is None else gI.contiguous(), None if gR is None else gR.contiguous(),
            params=dict(rho=rho.detach().contiguous(), angle_exp=k.detach().contiguous(),
                        pose_delta=pose_delta.detach().contiguous()), intensity=inten)
        return None, d_rho, d_k, d_pose, None, None


class LidarSpectralReturn(torch.autograd.Function):
    """(spectra[nmat, nbins], k[nmat], pose_delta[6]) -> (intensity, range, valid, tri) of one
    scan at the context's sensor wavelength (noise as in LidarReturn).

    R_lambda(0) is read from `spectra` at the wavelength (linear between bins),
    so the backward pass (the library's full-spectrum adjoint, hit triangles
    fixed) gives gradient to the one or two bins around it; scans at several
    wavelengths, each through its own call, add up in autograd.
    """

    @staticmethod
    def forward(ctx_, lidar_ctx: Context, spectra, k, pose_delta, seed: int = 0, scan: int = 0):
        prm = dict(spectra=spectra.detach().contiguous(), angle_exp=k.detach().contiguous(),
                   pose_delta=pose_delta.detach().contiguous())
        out = lidar_ctx.simulate(seed, scan, out=alloc_outputs(lidar_ctx.n_beams, ("intensity", "range", "valid",
                                                                                  "tri"), lidar_ctx.device),
                                 params=prm)
        ctx_.lidar = lidar_ctx
        ctx_.save_for_backward(spectra, k, pose_delta, out["tri"], out["valid"], out["intensity"])
        ctx_.mark_non_differentiable(out["valid"], out["tri"])
        return out["intensity"], out["range"], out["valid"], out["tri"]

    @staticmethod
    def backward(ctx_, gI, gR, _gv, _gt):
        spectra, k, pose_delta, tri, valid, inten = ctx_.saved_tensors
        d_T, d_k, d_pose = ctx_.lidar.backward_spectra(
            tri, valid, None if gI is None else gI.contiguous(), None if gR is None else gR.contiguous(),
            params=dict(spectra=spectra.detach().contiguous(), angle_exp=k.detach().contiguous(),
                        pose_delta=pose_delta.detach().contiguous()), intensity=inten)
        return None, d_T, d_k, d_pose, None, None
