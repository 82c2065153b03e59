"""Seeded synthetic scenes, sensors, poses and instance lists.

This module is the only code shared by the GPU path's tests/benchmark and the
oracle.  It builds geometry (FP32 vertices, u32 indices), per-triangle material
ids and instance labels, per-material spectral tables, sensor descriptions
(channel elevations in degrees, azimuth count) and poses.  It contains none of
the LiDAR method's arithmetic: no beam directions, no intersection, no return
model, no noise.

Workloads (stand-ins for the paper's Unreal scenes, which are not available):

* ``small_16ch``: 16-channel sensor at 1.5 m over a 200 m x 200 m ground plane with
  20 boxes and 10 UV spheres (1,202 triangles, 4 materials, 31 labels).
* ``urban_64ch``: 64-channel sensor (non-uniform elevations, denser at the
  horizon), 2048 azimuth steps, in a procedural urban scene of 522,272
  triangles (terrain 256 x 256 cells, 400 buildings, 2,000 poles, 200 cars).
* ``urban_sequence_128ch``: 128-channel x 1024 sensor, 100 poses along a 10 Hz spline
  trajectory through the urban generator scaled 10x in area (5,224,200
  triangles, 64 materials).
* ``batch_256``: 256 sensor instances of four beam layouts at random road poses
  in the urban_64ch scene.
* ``calibration_20mat``: urban_64ch geometry with 20 materials and hidden per-material
  reflectance / angle exponent / pose for calibration.
* ``dynamic_actors``: the urban_64ch scene plus 200 moving cars (three car meshes)
  and 100 walking, deforming pedestrians placed by rigid transforms.

The spectral tables stand in for the ECOSTRESS library (paper, Section II-C):
61 bins from 400 nm to 1000 nm in 10 nm steps, values i.i.d. U(0.05, 0.9)
smoothed with a [1,2,3,2,1]/9 kernel (edge replication).
"""
from __future__ import annotations

import functools
import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

N_BINS = 61
LAMBDA0_NM = 400.0
DLAMBDA_NM = 10.0
ROAD_PITCH = 64.0
ROAD_HALF = 5.0


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class Scene:
    vertices: np.ndarray          # float32 [nv, 3]
    indices: np.ndarray           # uint32 [nt, 3]
    material: np.ndarray          # uint16 [nt]
    label: np.ndarray             # uint32 [nt]
    spectra: np.ndarray           # float32 [nmat, 61] reflectance at 0 deg incidence
    sigma_range: np.ndarray       # float32 [nmat] Gaussian range-noise sigma (m)
    angle_exp: np.ndarray         # float32 [nmat] exponent k of cos^k (1 = Lambertian)
    heights: object = None        # terrain height function h(x, y) (float64) or None
    objects: list = field(default_factory=list)  # AABBs of placed objects (x0,y0,x1,y1)

    @property
    def n_tri(self) -> int:
        return int(self.indices.shape[0])

    @property
    def nmat(self) -> int:
        return int(self.spectra.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.vertices, self.indices, self.material, self.label,
                  self.spectra, self.sigma_range, self.angle_exp):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


@dataclass
class Sensor:
    elev_deg: np.ndarray          # float64 [n_ch] channel elevations
    n_az: int                     # azimuth samples over fov_h
    az0_deg: float = 0.0
    fov_h_deg: float = 360.0
    wavelength_nm: float = 905.0
    d_max: float = 100.0          # maximum range (m)
    r_l_max: float = 0.80         # reflectance needed at d_max (fraction)
    t_min: float = 0.01           # minimum range (m)
    sigma_intensity: float = 0.0  # additive intensity noise sigma
    noise_on: bool = True

    def __post_init__(self):
        # the library's sensor descriptor carries these as float32; keep the
        # values exactly representable so both consumers see the same numbers
        for k in ("wavelength_nm", "d_max", "r_l_max", "t_min", "sigma_intensity"):
            setattr(self, k, float(np.float32(getattr(self, k))))
        self.elev_deg = np.asarray(self.elev_deg, dtype=np.float64)

    @property
    def n_ch(self) -> int:
        return int(len(self.elev_deg))

    @property
    def n_beams(self) -> int:
        return self.n_ch * self.n_az


@dataclass
class Pose:
    p: np.ndarray                 # float32 [3] sensor origin (world)
    q: np.ndarray                 # float32 [4] orientation quaternion (w, x, y, z)


@dataclass
class Instance:
    sensor: Sensor
    pose: Pose
    seed: int = 0
    scan: int = 0


# ----------------------------------------------------------------------------
# channel elevation tables (data-sheet style), degrees
# ----------------------------------------------------------------------------
def elev_uniform(n: int, lo: float, hi: float) -> np.ndarray:
    return np.linspace(lo, hi, n, dtype=np.float64)


def elev_sinh64() -> np.ndarray:
    """64 channels from -25 to +15 deg, ~0.33 deg apart at the horizon, ~1.6 deg at the bottom."""
    a, b = math.asinh(-5.0), math.asinh(3.0)
    j = np.arange(64, dtype=np.float64)
    return 5.0 * np.sinh(a + j * (b - a) / 63.0)


def elev_table(n_ch: int) -> np.ndarray:
    if n_ch == 16:
        return elev_uniform(16, -15.0, 15.0)
    if n_ch == 32:
        return elev_uniform(32, -25.0, 15.0)
    if n_ch == 64:
        return elev_sinh64()
    if n_ch == 128:
        return elev_uniform(128, -45.0, 45.0)
    raise ValueError(f"no elevation table for {n_ch} channels")


# ----------------------------------------------------------------------------
# small helpers
# ----------------------------------------------------------------------------
def quat_from_ypr(yaw: float, pitch: float = 0.0, roll: float = 0.0) -> np.ndarray:
    """Quaternion (w, x, y, z) for intrinsic z-y-x (yaw, pitch, roll) angles in radians."""
    cy, sy = math.cos(yaw / 2), math.sin(yaw / 2)
    cp, sp = math.cos(pitch / 2), math.sin(pitch / 2)
    cr, sr = math.cos(roll / 2), math.sin(roll / 2)
    w = cr * cp * cy + sr * sp * sy
    x = sr * cp * cy - cr * sp * sy
    y = cr * sp * cy + sr * cp * sy
    z = cr * cp * sy - sr * sp * cy
    q = np.array([w, x, y, z], dtype=np.float64)
    return (q / np.linalg.norm(q)).astype(np.float32)


def spectra_table(rng: np.random.Generator, nmat: int) -> np.ndarray:
    raw = rng.uniform(0.05, 0.9, size=(nmat, N_BINS))
    k = np.array([1, 2, 3, 2, 1], dtype=np.float64) / 9.0
    padded = np.pad(raw, ((0, 0), (2, 2)), mode="edge")
    out = np.empty_like(raw)
    for i in range(N_BINS):
        out[:, i] = padded[:, i:i + 5] @ k
    return out.astype(np.float32)


class _MeshBuilder:
    def __init__(self):
        self.v, self.i, self.m, self.l = [], [], [], []
        self.nv = 0

    def add(self, verts: np.ndarray, tris: np.ndarray, mat: int, label: int):
        verts = np.asarray(verts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        self.v.append(verts)
        self.i.append(tris + self.nv)
        self.m.append(np.full(len(tris), mat, dtype=np.uint16))
        self.l.append(np.full(len(tris), label, dtype=np.uint32))
        self.nv += len(verts)

    def add_many(self, verts: np.ndarray, tris: np.ndarray, mats: np.ndarray, labels: np.ndarray):
        """verts [n_obj, nv_obj, 3], tris [nt_obj, 3] shared topology."""
        n_obj, nvo, _ = verts.shape
        off = self.nv + np.arange(n_obj, dtype=np.int64)[:, None, None] * nvo
        self.v.append(verts.reshape(-1, 3))
        self.i.append((tris[None, :, :] + off).reshape(-1, 3))
        self.m.append(np.repeat(np.asarray(mats, dtype=np.uint16), len(tris)))
        self.l.append(np.repeat(np.asarray(labels, dtype=np.uint32), len(tris)))
        self.nv += n_obj * nvo

    def finish(self):
        v = np.concatenate(self.v).astype(np.float32)
        i = np.concatenate(self.i).astype(np.uint32)
        m = np.concatenate(self.m)
        lab = np.concatenate(self.l)
        return v, i, m, lab


# unit box corners (0/1) and its 12 triangles
_BOX_CORNERS = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float64)
_BOX_TRIS = np.array([
    [0, 2, 1], [1, 2, 3],      # bottom z=0
    [4, 5, 6], [5, 7, 6],      # top z=1
    [0, 1, 4], [1, 5, 4],      # y=0
    [2, 6, 3], [3, 6, 7],      # y=1
    [0, 4, 2], [2, 4, 6],      # x=0
    [1, 3, 5], [3, 7, 5],      # x=1
], dtype=np.int64)


def box_mesh(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + _BOX_CORNERS * (hi - lo), _BOX_TRIS


def boxes_oriented(centers, half, yaw):
    """Many yawed boxes: centers [n,3] (base centre), half [n,3] (hx, hy, full height), yaw [n]."""
    c = np.cos(yaw)[:, None]
    s = np.sin(yaw)[:, None]
    loc = (_BOX_CORNERS[None] * 2.0 - 1.0) * half[:, None, :]
    loc[..., 2] = (_BOX_CORNERS[None, :, 2]) * half[:, None, 2]
    x = loc[..., 0] * c - loc[..., 1] * s
    y = loc[..., 0] * s + loc[..., 1] * c
    v = np.stack([x, y, loc[..., 2]], axis=-1) + centers[:, None, :]
    return v, _BOX_TRIS


def cylinder_topology(seg: int = 32, stacks: int = 2):
    """Vertex layout: (stacks+1) rings of `seg`, then bottom centre, top centre."""
    tris = []
    for s in range(stacks):
        for k in range(seg):
            a = s * seg + k
            b = s * seg + (k + 1) % seg
            c = (s + 1) * seg + k
            d = (s + 1) * seg + (k + 1) % seg
            tris += [[a, b, c], [b, d, c]]
    bc = (stacks + 1) * seg
    tc = bc + 1
    for k in range(seg):
        tris.append([bc, (k + 1) % seg, k])
        tris.append([tc, stacks * seg + k, stacks * seg + (k + 1) % seg])
    return np.array(tris, dtype=np.int64)


def cylinders(centers, radius, height, seg: int = 32, stacks: int = 2):
    ang = 2.0 * np.pi * np.arange(seg) / seg
    n = len(centers)
    zs = np.linspace(0.0, 1.0, stacks + 1)
    ring = np.stack([np.cos(ang), np.sin(ang)], axis=-1)             # [seg, 2]
    v = np.zeros((n, (stacks + 1) * seg + 2, 3))
    for s, zf in enumerate(zs):
        v[:, s * seg:(s + 1) * seg, 0:2] = ring[None] * radius[:, None, None]
        v[:, s * seg:(s + 1) * seg, 2] = (zf * height)[:, None]
    v[:, -1, 2] = height
    v += centers[:, None, :]
    return v, cylinder_topology(seg, stacks)


def uv_sphere_topology(seg: int, stacks: int):
    """Vertex layout: north pole, (stacks-1) rings of `seg`, south pole."""
    tris = []
    n_rings = stacks - 1
    south = 1 + n_rings * seg
    for k in range(seg):
        tris.append([0, 1 + k, 1 + (k + 1) % seg])
    for r in range(n_rings - 1):
        for k in range(seg):
            a = 1 + r * seg + k
            b = 1 + r * seg + (k + 1) % seg
            c = 1 + (r + 1) * seg + k
            d = 1 + (r + 1) * seg + (k + 1) % seg
            tris += [[a, c, b], [b, c, d]]
    base = 1 + (n_rings - 1) * seg
    for k in range(seg):
        tris.append([south, base + (k + 1) % seg, base + k])
    return np.array(tris, dtype=np.int64)


def uv_sphere(center, radius, seg: int, stacks: int):
    """UV sphere with `seg` segments and `stacks` stacks: 2*seg*(stacks-1) triangles."""
    verts = [[0.0, 0.0, 1.0]]
    for r in range(1, stacks):
        pol = math.pi * r / stacks
        for k in range(seg):
            az = 2.0 * math.pi * k / seg
            verts.append([math.sin(pol) * math.cos(az), math.sin(pol) * math.sin(az), math.cos(pol)])
    verts.append([0.0, 0.0, -1.0])
    v = np.asarray(center, dtype=np.float64) + radius * np.asarray(verts)
    return v, uv_sphere_topology(seg, stacks)


# ----------------------------------------------------------------------------
# config 1: ground + 20 boxes + 10 spheres
# ----------------------------------------------------------------------------
def _overlaps(box, placed, gap=0.5):
    x0, y0, x1, y1 = box
    for (a0, b0, a1, b1) in placed:
        if x0 < a1 + gap and x1 > a0 - gap and y0 < b1 + gap and y1 > b0 - gap:
            return True
    return False


def _near_origin(box, clear=2.0):
    x0, y0, x1, y1 = box
    dx = max(x0, -x1, 0.0)
    dy = max(y0, -y1, 0.0)
    return math.hypot(dx, dy) < clear


@functools.lru_cache(maxsize=4)
def small_16ch(seed: int = 1001):
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    nmat = 4
    # ground [-100, 100]^2 at z = 0: two triangles, material 0, label 1
    gv = np.array([[-100, -100, 0], [100, -100, 0], [100, 100, 0], [-100, 100, 0]], dtype=np.float64)
    mb.add(gv, np.array([[0, 1, 2], [0, 2, 3]]), 0, 1)
    placed = []
    label = 2
    while len(placed) < 20:
        size = rng.uniform(1.0, 8.0, size=3)
        c = rng.uniform(-50.0, 50.0, size=2)
        box = (c[0] - size[0] / 2, c[1] - size[1] / 2, c[0] + size[0] / 2, c[1] + size[1] / 2)
        if _overlaps(box, placed) or _near_origin(box):
            continue
        placed.append(box)
        v, t = box_mesh([box[0], box[1], 0.0], [box[2], box[3], size[2]])
        mb.add(v, t, int(rng.integers(0, nmat)), label)
        label += 1
    n_sph = 0
    while n_sph < 10:
        r = rng.uniform(0.5, 3.0)
        c = rng.uniform(-50.0, 50.0, size=2)
        box = (c[0] - r, c[1] - r, c[0] + r, c[1] + r)
        if _overlaps(box, placed) or _near_origin(box):
            continue
        placed.append(box)
        v, t = uv_sphere([c[0], c[1], r], r, 8, 7)
        mb.add(v, t, int(rng.integers(0, nmat)), label)
        label += 1
        n_sph += 1
    v, i, m, lab = mb.finish()
    scene = Scene(v, i, m, lab, spectra_table(rng, nmat),
                  np.full(nmat, 0.02, np.float32), np.ones(nmat, np.float32),
                  heights=lambda x, y: np.zeros_like(np.asarray(x, dtype=np.float64)),
                  objects=placed)
    sensor = Sensor(elev_table(16), 900, wavelength_nm=905.0, d_max=100.0)
    pose = Pose(np.array([0.0, 0.0, 1.5], np.float32), np.array([1, 0, 0, 0], np.float32))
    return scene, sensor, pose


# ----------------------------------------------------------------------------
# urban generator (configs 2-5)
# ----------------------------------------------------------------------------
def _terrain_fn(rng: np.random.Generator, half_extent: float, amp: float = 1.5):
    n = 6
    wl = rng.uniform(60.0, 300.0, size=n)
    ang = rng.uniform(0.0, 2 * np.pi, size=n)
    ph = rng.uniform(0.0, 2 * np.pi, size=n)
    a = rng.uniform(0.5, 1.0, size=n)
    kx = 2 * np.pi / wl * np.cos(ang)
    ky = 2 * np.pi / wl * np.sin(ang)
    scale = amp / a.sum()

    def h(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for j in range(n):
            out = out + a[j] * np.sin(kx[j] * x + ky[j] * y + ph[j])
        return out * scale
    return h


def _terrain_mesh(cells: int, cell: float, h):
    half = cells * cell / 2.0
    xs = np.linspace(-half, half, cells + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    Z = h(X, Y)
    v = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    r = np.arange(cells)
    i00 = (r[:, None] * (cells + 1) + r[None, :]).reshape(-1)   # row=y index, col=x index
    i10 = i00 + 1
    i01 = i00 + (cells + 1)
    i11 = i01 + 1
    t1 = np.stack([i00, i10, i11], axis=-1)
    t2 = np.stack([i00, i11, i01], axis=-1)
    t = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return v, t


def _on_road(x0, y0, x1, y1):
    for a0, a1 in ((x0, x1), (y0, y1)):
        k0 = math.floor((a0 - ROAD_HALF) / ROAD_PITCH)
        k1 = math.ceil((a1 + ROAD_HALF) / ROAD_PITCH)
        for k in range(k0, k1 + 1):
            c = k * ROAD_PITCH
            if a0 < c + ROAD_HALF and a1 > c - ROAD_HALF:
                return True
    return False


class _Grid:
    """Spatial hash of placed AABBs (x0, y0, x1, y1) for overlap rejection."""

    def __init__(self, cell=32.0):
        self.cell = cell
        self.cells = {}
        self.boxes = []

    def _keys(self, b):
        c = self.cell
        for i in range(math.floor(b[0] / c), math.floor(b[2] / c) + 1):
            for j in range(math.floor(b[1] / c), math.floor(b[3] / c) + 1):
                yield (i, j)

    def hit(self, b, gap=0.5):
        g = (b[0] - gap, b[1] - gap, b[2] + gap, b[3] + gap)
        for k in self._keys(g):
            for idx in self.cells.get(k, ()):
                a = self.boxes[idx]
                if g[0] < a[2] and g[2] > a[0] and g[1] < a[3] and g[3] > a[1]:
                    return True
        return False

    def add(self, b):
        self.boxes.append(b)
        for k in self._keys(b):
            self.cells.setdefault(k, []).append(len(self.boxes) - 1)


def urban_scene(seed: int, cells: int, n_build: int, n_poles: int, n_cars: int, nmat: int,
                mat_seed: int | None = None) -> Scene:
    """Procedural urban scene: terrain + buildings + poles + cars.

    Geometry depends only on `seed`; material ids are drawn from a separate
    stream (`mat_seed`) so that scenes differing only in their material count
    share their triangles.  Labels: terrain 1, then objects 2, 3, ...
    """
    rng = np.random.default_rng(seed)
    cell = 2.0
    half = cells * cell / 2.0
    h = _terrain_fn(rng, half)
    grid = _Grid()
    margin = 8.0
    lo, hi = -half + margin, half - margin

    # buildings: axis-aligned footprint U(6, 20), height U(4, 40), sunk 2 m
    bld = []
    while len(bld) < n_build:
        fx, fy = rng.uniform(6.0, 20.0, size=2)
        cx, cy = rng.uniform(lo, hi, size=2)
        b = (cx - fx / 2, cy - fy / 2, cx + fx / 2, cy + fy / 2)
        if _on_road(*b) or grid.hit(b):
            continue
        grid.add(b)
        bld.append((b, rng.uniform(4.0, 40.0)))
    # poles near road edges: r U(0.08, 0.3), height U(3, 10)
    poles = []
    while len(poles) < n_poles:
        r = rng.uniform(0.08, 0.3)
        ht = rng.uniform(3.0, 10.0)
        k = rng.integers(math.ceil(lo / ROAD_PITCH), math.floor(hi / ROAD_PITCH) + 1)
        along = rng.uniform(lo, hi)
        off = rng.choice([-1.0, 1.0]) * rng.uniform(5.5, 7.5)
        if rng.integers(0, 2) == 0:
            cx, cy = k * ROAD_PITCH + off, along
        else:
            cx, cy = along, k * ROAD_PITCH + off
        b = (cx - r, cy - r, cx + r, cy + r)
        if _on_road(*b) or grid.hit(b, gap=0.3):
            continue
        grid.add(b)
        poles.append((cx, cy, r, ht))
    # cars on road lanes, >= 8 m from the origin
    cars = []
    while len(cars) < n_cars:
        L, W, H = np.array([4.5, 1.8, 1.5]) * rng.uniform(0.9, 1.1, size=3)
        k = rng.integers(math.ceil(lo / ROAD_PITCH), math.floor(hi / ROAD_PITCH) + 1)
        along = rng.uniform(lo, hi)
        lane = rng.choice([-2.5, 2.5])
        if rng.integers(0, 2) == 0:
            cx, cy, yaw = k * ROAD_PITCH + lane, along, math.pi / 2 + rng.uniform(-0.05, 0.05)
        else:
            cx, cy, yaw = along, k * ROAD_PITCH + lane, rng.uniform(-0.05, 0.05)
        if rng.integers(0, 2):
            yaw += math.pi
        ext = 0.5 * (abs(L * math.cos(yaw)) + abs(W * math.sin(yaw)))
        eyt = 0.5 * (abs(L * math.sin(yaw)) + abs(W * math.cos(yaw)))
        b = (cx - ext, cy - eyt, cx + ext, cy + eyt)
        if math.hypot(cx, cy) < 8.0 or grid.hit(b, gap=1.0):
            continue
        grid.add(b)
        cars.append((cx, cy, L, W, H, yaw))

    mrng = np.random.default_rng(seed * 7919 + 17 if mat_seed is None else mat_seed)
    n_obj = n_build + n_poles + n_cars
    obj_mat = mrng.integers(0, nmat, size=n_obj)
    spectra = spectra_table(mrng, nmat)

    mb = _MeshBuilder()
    tv, tt = _terrain_mesh(cells, cell, h)
    mb.add(tv, tt, int(mrng.integers(0, nmat)), 1)
    label = 2
    # buildings (shared box topology)
    bb = np.array([b for b, _ in bld])
    bh = np.array([ht for _, ht in bld])
    cx = (bb[:, 0] + bb[:, 2]) / 2
    cy = (bb[:, 1] + bb[:, 3]) / 2
    z0 = h(cx, cy) - 2.0
    lo3 = np.stack([bb[:, 0], bb[:, 1], z0], -1)
    hi3 = np.stack([bb[:, 2], bb[:, 3], z0 + 2.0 + bh], -1)
    v = lo3[:, None, :] + _BOX_CORNERS[None] * (hi3 - lo3)[:, None, :]
    mb.add_many(v, _BOX_TRIS, obj_mat[:n_build], np.arange(label, label + n_build))
    label += n_build
    # poles
    pa = np.array(poles)
    pz = h(pa[:, 0], pa[:, 1]) - 0.5
    v, t = cylinders(np.stack([pa[:, 0], pa[:, 1], pz], -1), pa[:, 2], pa[:, 3] + 0.5)
    mb.add_many(v, t, obj_mat[n_build:n_build + n_poles], np.arange(label, label + n_poles))
    label += n_poles
    # cars
    ca = np.array(cars)
    cz = h(ca[:, 0], ca[:, 1]) - 0.2
    v, t = boxes_oriented(np.stack([ca[:, 0], ca[:, 1], cz], -1),
                          np.stack([ca[:, 2] / 2, ca[:, 3] / 2, ca[:, 4] + 0.2], -1), ca[:, 5])
    mb.add_many(v, t, obj_mat[n_build + n_poles:], np.arange(label, label + n_cars))
    label += n_cars

    v, i, m, lab = mb.finish()
    return Scene(v, i, m, lab, spectra, np.full(nmat, 0.02, np.float32),
                 np.ones(nmat, np.float32), heights=h, objects=list(grid.boxes))


@functools.lru_cache(maxsize=4)
def urban_small(nmat: int = 32, seed: int = 2002) -> Scene:
    """The ~500k-triangle urban scene (256 x 256 terrain cells)."""
    return urban_scene(seed, 256, 400, 2000, 200, nmat, mat_seed=seed * 31 + nmat)


@functools.lru_cache(maxsize=1)
def urban_large(nmat: int = 64, seed: int = 3003) -> Scene:
    """The ~5.2M-triangle urban scene (10x area: 810 x 810 cells)."""
    return urban_scene(seed, 810, 4000, 20000, 2000, nmat, mat_seed=seed * 31 + nmat)


def _sensor_pose_at(scene: Scene, x: float, y: float, yaw: float = 0.0, pitch=0.0, roll=0.0,
                    height: float = 1.8) -> Pose:
    z = float(scene.heights(x, y)) + height
    return Pose(np.array([x, y, z], np.float32), quat_from_ypr(yaw, pitch, roll))


def urban_64ch(seed: int = 2002):
    scene = urban_small(32, seed)
    sensor = Sensor(elev_table(64), 2048, wavelength_nm=905.0, d_max=100.0)
    return scene, sensor, _sensor_pose_at(scene, 0.0, 0.0)


def catmull_rom(points: np.ndarray, samples_per_seg: int = 200) -> np.ndarray:
    P = np.asarray(points, dtype=np.float64)
    P = np.vstack([2 * P[0] - P[1], P, 2 * P[-1] - P[-2]])
    out = []
    for k in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[k - 1], P[k], P[k + 1], P[k + 2]
        s = np.linspace(0, 1, samples_per_seg, endpoint=False)[:, None]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s ** 2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * s ** 3))
    out.append(P[-2][None])
    return np.vstack(out)


def trajectory(scene: Scene, seed: int, n: int = 100, speed: float = 10.0, rate_hz: float = 10.0):
    """Poses at `rate_hz` along a Catmull-Rom spline through road control points."""
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-1.0, 1.0, size=(8, 2)) * np.array([[0.0, 1.0]] * 4 + [[1.0, 0.0]] * 4)
    ctrl = np.array([[-70, 0], [-50, 0], [-30, 0], [-10, 0], [0, 10], [0, 30], [0, 50], [0, 70]],
                    dtype=np.float64) + jit
    curve = catmull_rom(ctrl)
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    s0 = 0.5 * (s[-1] - speed * (n - 1) / rate_hz)
    poses = []
    for k in range(n):
        sk = s0 + speed * k / rate_hz
        x = np.interp(sk, s, curve[:, 0])
        y = np.interp(sk, s, curve[:, 1])
        x2 = np.interp(sk + 0.5, s, curve[:, 0])
        y2 = np.interp(sk + 0.5, s, curve[:, 1])
        poses.append(_sensor_pose_at(scene, x, y, math.atan2(y2 - y, x2 - x)))
    return poses


def urban_sequence_128ch(seed: int = 3003):
    scene = urban_large(64, seed)
    sensor = Sensor(elev_table(128), 1024, wavelength_nm=905.0, d_max=100.0, sigma_intensity=0.01)
    return scene, sensor, trajectory(scene, seed + 1)


def batch_256(seed: int = 4004, n_inst: int = 256):
    """256 instances, 1:1:1:1 of 16x900, 32x1800, 64x2048, 128x1024, at random road poses."""
    scene = urban_small(32, 2002)
    rng = np.random.default_rng(seed)
    kinds = np.array([(16, 900), (32, 1800), (64, 2048), (128, 1024)] * (n_inst // 4))
    kinds = kinds[rng.permutation(len(kinds))]
    half = 256.0 - 20.0
    insts = []
    for j, (nch, naz) in enumerate(kinds):
        while True:
            along = rng.uniform(-half, half)
            k = rng.integers(-3, 4)
            off = rng.uniform(-3.0, 3.0)
            if rng.integers(0, 2):
                x, y = k * ROAD_PITCH + off, along
            else:
                x, y = along, k * ROAD_PITCH + off
            inside = any(b[0] - 1 < x < b[2] + 1 and b[1] - 1 < y < b[3] + 1 for b in scene.objects)
            if not inside:
                break
        yaw = rng.uniform(0, 2 * math.pi)
        pitch, roll = np.deg2rad(rng.uniform(-3, 3, size=2))
        lam = float(rng.choice([850.0, 905.0, 1550.0]))
        dmax = float(rng.uniform(50.0, 200.0))
        sensor = Sensor(elev_table(int(nch)), int(naz), wavelength_nm=lam, d_max=dmax)
        insts.append(Instance(sensor, _sensor_pose_at(scene, x, y, yaw, pitch, roll), seed=seed, scan=0))
    return scene, insts


def calibration_20mat(seed: int = 5005):
    """Calibration problem: 20 materials, hidden (rho*, k*, pose*), perturbed start."""
    scene = urban_small(20, 2002)
    rng = np.random.default_rng(seed)
    rho_true = rng.uniform(0.05, 0.9, size=20).astype(np.float32)
    k_true = rng.uniform(0.5, 2.5, size=20).astype(np.float32)
    sensor = Sensor(elev_table(64), 2048, wavelength_nm=905.0, d_max=100.0, noise_on=False)
    pose_true = _sensor_pose_at(scene, 0.0, 0.0, yaw=float(rng.uniform(0, 2 * math.pi)))
    dp = rng.uniform(-0.2, 0.2, size=3)
    dang = np.deg2rad(rng.uniform(-1.0, 1.0, size=3))
    return dict(scene=scene, sensor=sensor, pose_true=pose_true, rho_true=rho_true, k_true=k_true,
                dp0=dp, dw0=dang, rho0=np.full(20, 0.3, np.float32), k0=np.ones(20, np.float32))


# ----------------------------------------------------------------------------
# dynamic scenes: meshes placed by moving actors
# ----------------------------------------------------------------------------
@dataclass
class Mesh:
    vertices: np.ndarray          # float32 [nv, 3], object space
    indices: np.ndarray           # uint32 [nt, 3]
    material: np.ndarray          # uint16 [nt]

    @property
    def n_tri(self) -> int:
        return int(self.indices.shape[0])


@dataclass
class Actor:
    mesh: int                     # index into the mesh list
    label: int                    # instance label of every triangle of this actor
    p: np.ndarray                 # float32 [3] object origin in the world
    q: np.ndarray                 # float32 [4] orientation (w, x, y, z)


def _wheel(cx, cy, r, w, seg=24):
    """Cylinder with its axis along y, centre (cx, cy, r): ring vertices then the two cap centres."""
    ang = 2.0 * np.pi * np.arange(seg) / seg
    v = []
    for y in (cy - w / 2, cy + w / 2):
        for a in ang:
            v.append([cx + r * math.cos(a), y, r + r * math.sin(a)])
    v.append([cx, cy - w / 2, r])
    v.append([cx, cy + w / 2, r])
    return np.array(v), cylinder_topology(seg, 1)


def _assemble(parts):
    vs, ts, ms = [], [], []
    base = 0
    for v, t, m in parts:
        vs.append(np.asarray(v, np.float64))
        ts.append(np.asarray(t, np.int64) + base)
        ms.append(np.full(len(t), m, np.uint16))
        base += len(v)
    return Mesh(np.concatenate(vs).astype(np.float32), np.concatenate(ts).astype(np.uint32), np.concatenate(ms))


def car_mesh(length=4.5, width=1.8, height=1.5, mats=(3, 7, 11)):
    """A car in object space (x forward, base at z = 0): body, cabin and four wheels; 408 triangles."""
    L, W, H = length, width, height
    parts = []
    v, t = box_mesh([-L / 2, -W / 2, 0.3], [L / 2, W / 2, 0.3 + 0.55 * H])
    parts.append((v, t, mats[0]))
    v, t = box_mesh([-0.3 * L, -0.45 * W, 0.3 + 0.55 * H], [0.25 * L, 0.45 * W, H])
    parts.append((v, t, mats[1]))
    for sx in (-0.32 * L, 0.32 * L):
        for sy in (-W / 2 + 0.11, W / 2 - 0.11):
            v, t = _wheel(sx, sy, 0.33, 0.22)
            parts.append((v, t, mats[2]))
    return _assemble(parts)


def pedestrian_mesh(mats=(5, 9)):
    """A pedestrian in object space: torso cylinder and head sphere; 304 triangles."""
    v, t = cylinders(np.array([[0.0, 0.0, 0.0]]), np.array([0.2]), np.array([1.45]), seg=16, stacks=4)
    parts = [(v[0], t, mats[0])]
    v, t = uv_sphere([0.0, 0.0, 1.6], 0.13, 12, 7)
    parts.append((v, t, mats[1]))
    return _assemble(parts)


def pedestrian_pose_vertices(mesh: Mesh, phase: float) -> np.ndarray:
    """Deformed (walking sway) object-space vertices of ``pedestrian_mesh``, same topology."""
    v = mesh.vertices.astype(np.float64).copy()
    z = v[:, 2] / 1.75
    v[:, 0] += 0.15 * math.sin(phase) * z * z
    v[:, 1] += 0.05 * math.cos(phase) * z
    return v.astype(np.float32)


def dynamic_actors(seed: int = 6006, n_cars: int = 200, n_peds: int = 100):
    """Moving actors in the 522k-triangle urban scene.

    Three car meshes (408 triangles each) and one deformable pedestrian mesh
    (304 triangles); cars drive along the road lanes at U(5, 15) m/s,
    pedestrians walk along the sidewalks at 1.4 m/s.  Returns a dict with the
    static scene, sensor, sensor pose, meshes, and ``actors_at(t)`` giving the
    actor list at time t (labels 100000 + k).
    """
    scene = urban_small(32, 2002)
    _, sensor, pose = urban_64ch()
    meshes = [car_mesh(4.5, 1.8, 1.5), car_mesh(4.0, 1.7, 1.45, mats=(4, 7, 11)),
              car_mesh(5.2, 2.0, 1.9, mats=(13, 7, 11)), pedestrian_mesh()]
    rng = np.random.default_rng(seed)
    half = 256 * 2.0 / 2.0 - 8.0
    kmin, kmax = math.ceil(-half / ROAD_PITCH), math.floor(half / ROAD_PITCH)
    specs = []
    for k in range(n_cars + n_peds):
        car = k < n_cars
        road = int(rng.integers(kmin, kmax + 1))
        axis = int(rng.integers(0, 2))             # 0: road along y (x = const), 1: along x
        side = float(rng.choice([-1.0, 1.0]))
        off = side * (2.5 if car else 6.5)
        along0 = float(rng.uniform(-half, half))
        speed = float(rng.uniform(5.0, 15.0)) if car else 1.4
        # right-hand traffic: the lane at +offset drives in +direction
        direction = side
        mesh = int(rng.integers(0, 3)) if car else 3
        # keep the origin clearing free at t = 0
        if abs(along0) < 12.0 and abs(road) == 0:
            along0 += 24.0
        specs.append((mesh, road * ROAD_PITCH + off, axis, along0, speed * direction))

    def actors_at(t: float):
        out = []
        for k, (mesh, c, axis, a0, v) in enumerate(specs):
            a = a0 + v * t
            a = (a + half) % (2 * half) - half     # wrap inside the scene
            x, y = (c, a) if axis == 0 else (a, c)
            yaw = (math.pi / 2 if axis == 0 else 0.0) + (0.0 if v >= 0 else math.pi)
            z = float(scene.heights(x, y)) - (0.05 if mesh < 3 else 0.0)
            out.append(Actor(mesh, 100000 + k, np.array([x, y, z], np.float32), quat_from_ypr(yaw)))
        return out

    return dict(scene=scene, sensor=sensor, pose=pose, meshes=meshes, actors_at=actors_at)
