"""FP64 reference implementation of the per-beam LiDAR return (TEST INFRASTRUCTURE ONLY).

This is the oracle: plain, slow, double-precision code that states what the
simulation computes, step by step in the order of the paper (Jansen, Huebel,
Steckel, "Physical LiDAR Simulation in Real-Time Engine", arXiv:2208.10295).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU library and imports nothing from it; the
two meet only in the seeded inputs of ``lidar_inputs``.

Steps (paper section in brackets):

1. Beam pattern [II-A, eq.3 and the text after it]: azimuth theta_i spans
   FOV_h in equal steps, elevations phi_j come from the sensor's table.  The
   beam direction in the sensor frame is
   s = (cos phi cos theta, cos phi sin theta, sin phi); this is the direction
   whose pinhole projection gives eq.3 (tan theta horizontally,
   sin phi / (cos phi cos theta) vertically).  World ray: o = p, d = R s.
2. Depth [II-A]: the range of the first surface along the beam.  Computed as
   the first ray/triangle intersection (``first_hit.c``).
3. Labels [II-B]: the instance label of the object that owns the hit surface.
4. Material model [II-C, eq.4]: R_lambda(theta) = R_lambda(0) cos(theta), with
   cos(theta) from the dot product of the surface normal and the beam, and
   R_lambda(0) the material's spectral reflectance at the sensor wavelength.
   Generalised to cos^k with a per-material exponent k (k = 1 is eq.4).
5. Range noise [II-A, last paragraph]: Gaussian noise with a per-material
   scale sigma is added to the depth.  The Gaussian comes from a counter-based
   generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
   seed, counter (beam, scan, instance, 0), then Box-Muller.
6. Capability model [II-D, eq.5]: R_L(d) = R_L,max / d_max * d; the point is
   kept iff R_L(d) <= R_lambda, with d including the noise, and anything beyond
   d_max is dropped.
7. Output [Fig.1 caption]: a point cloud with depth, intensity and instance
   label per point.

Readings of points where the paper is silent or garbled are listed with the
functions that depend on them.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfirst_hit.so")
_lib = None

MISS_LABEL = 0xFFFFFFFF
MISS_TRI = 0xFFFFFFFF
# |z| of a Box-Muller normal from 32-bit uniforms is at most sqrt(-2 ln 2^-32) = 6.66043...
BOX_MULLER_BOUND = 6.6605
TIE_MARGIN_M = 1e-6          # second-hit margin below which a ray is ambiguous
EDGE_ABS_M = 1e-6            # edge-graze margin: EDGE_ABS_M + EDGE_REL * t
EDGE_REL = 1e-6


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_first_hit.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, P,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, P, P, P, P, P]
        lib.oracle_first_hit.restype = ctypes.c_int
        lib.oracle_first_hit_d.argtypes = lib.oracle_first_hit.argtypes
        lib.oracle_first_hit_d.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# ----------------------------------------------------------------------------
# step 1: beam pattern [II-A]
# ----------------------------------------------------------------------------
def beam_angles(sensor):
    """(theta [n_az], phi [n_ch]) in radians.

    theta_i = az0 + i * FOV_h / N_az (FOV_h usually 0..360 deg, Section II-A);
    phi_j = the data-sheet elevation of channel j.  Reading: azimuth 0 is the
    sensor x axis and grows counter-clockwise (right-handed, z up).
    """
    i = np.arange(sensor.n_az, dtype=np.float64)
    theta = np.deg2rad(sensor.az0_deg + i * (sensor.fov_h_deg / sensor.n_az))
    phi = np.deg2rad(np.asarray(sensor.elev_deg, dtype=np.float64))
    return theta, phi


def beam_directions(sensor) -> np.ndarray:
    """Unit beam directions in the sensor frame, [n_ch, n_az, 3], beam b = j * n_az + i."""
    theta, phi = beam_angles(sensor)
    cp, sp = np.cos(phi)[:, None], np.sin(phi)[:, None]
    ct, st = np.cos(theta)[None, :], np.sin(theta)[None, :]
    return np.stack([cp * ct, cp * st, np.broadcast_to(sp, (len(phi), len(theta)))], axis=-1)


def pixel_of_beam(theta, phi, width, fov_c):
    """Eq.1-3: pixel of beam (theta, phi) in a square pinhole camera of width W.

    f = W / (2 tan(FOV_c / 2)), c_u = c_v = W / 2 (eq.2).  The printed eq.3 for
    n_y is garbled ("(sin phi - f_y)" and "c_y"); it is read as the pinhole
    projection n_y = -f sin(phi) / (cos(phi) cos(theta)) + c_v.
    """
    f = width / (2.0 * math.tan(fov_c / 2.0))
    c = width / 2.0
    nx = math.sin(theta) * f / math.cos(theta) + c
    ny = -f * math.sin(phi) / (math.cos(phi) * math.cos(theta)) + c
    return nx, ny


def rotation_from_quat(q) -> np.ndarray:
    """Rotation matrix of the unit quaternion (w, x, y, z), FP64 (q normalised first)."""
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(np.asarray(q, dtype=np.float64))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def so3_exp(w) -> np.ndarray:
    """Rodrigues' formula: rotation by angle |w| about w / |w|."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def so3_left_jacobian(w) -> np.ndarray:
    """J_l(w) with Exp(w + e) = Exp(J_l(w) e) Exp(w) to first order in e."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-8:
        return np.eye(3) + 0.5 * K + K @ K / 6.0
    return np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K


# ----------------------------------------------------------------------------
# step 2: first hit (delegated to first_hit.c)
# ----------------------------------------------------------------------------
def first_hit(scene, orig, dirs, t_min, t_max):
    """Brute-force FP64 first hit of rays (orig[n,3], dirs[n,3]) against every triangle.

    Returns dict of arrays: tri (int64, -1 = none), t, t_second, edge_in, near_t.
    """
    lib = _load()
    orig = np.ascontiguousarray(np.broadcast_to(orig, dirs.shape), dtype=np.float64)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    n = dirs.shape[0]
    # FP64 vertices (actors placed by a rigid transform) are used as given; FP32 ones are promoted
    f64 = np.asarray(scene.vertices).dtype == np.float64
    vtx = np.ascontiguousarray(scene.vertices, dtype=np.float64 if f64 else np.float32)
    idx = np.ascontiguousarray(scene.indices, dtype=np.uint32)
    out = dict(tri=np.empty(n, np.int64), t=np.empty(n), t_second=np.empty(n),
               edge_in=np.empty(n), near_t=np.empty(n))
    fn = lib.oracle_first_hit_d if f64 else lib.oracle_first_hit
    rc = fn(n, orig.ctypes.data, dirs.ctypes.data, idx.shape[0], vtx.ctypes.data,
                              idx.ctypes.data, float(t_min), float(t_max), EDGE_ABS_M, EDGE_REL,
                              out["tri"].ctypes.data, out["t"].ctypes.data, out["t_second"].ctypes.data,
                              out["edge_in"].ctypes.data, out["near_t"].ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_first_hit allocation failed")
    return out


def face_normals(scene, tri) -> np.ndarray:
    """Geometric unit normal normalize((v1 - v0) x (v2 - v0)) of triangles `tri`, FP64."""
    v = scene.vertices.astype(np.float64)[scene.indices[tri].astype(np.int64)]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


# ----------------------------------------------------------------------------
# step 4: spectral reflectance at the sensor wavelength [II-C]
# ----------------------------------------------------------------------------
def reflectance_at_wavelength(spectra, wavelength_nm, lambda0_nm=400.0, dlambda_nm=10.0):
    """R_lambda(0 deg) per material at the sensor wavelength.

    Reading: linear interpolation between the 10-nm bins, clamped to the first
    and last bin outside the table (returns (R0[nmat], clamped_flag)).
    """
    T = np.asarray(spectra, dtype=np.float64)
    nb = T.shape[1]
    q = (float(wavelength_nm) - lambda0_nm) / dlambda_nm
    if q <= 0.0:
        return T[:, 0].copy(), q < 0.0
    if q >= nb - 1:
        return T[:, nb - 1].copy(), q > nb - 1
    i = int(math.floor(q))
    f = q - i
    return (1.0 - f) * T[:, i] + f * T[:, i + 1], False


def spectral_weights(nbins, wavelength_nm, lambda0_nm=400.0, dlambda_nm=10.0) -> np.ndarray:
    """w[nbins] such that R_lambda(0) = T w for every material row T: the linear
    interpolation weights of ``reflectance_at_wavelength`` ((1 - f) on bin i,
    f on bin i + 1; all weight on the end bin outside the table)."""
    w = np.zeros(nbins)
    q = (float(wavelength_nm) - lambda0_nm) / dlambda_nm
    if q <= 0.0:
        w[0] = 1.0
    elif q >= nbins - 1:
        w[nbins - 1] = 1.0
    else:
        i = int(math.floor(q))
        f = q - i
        w[i] = 1.0 - f
        w[i + 1] = f
    return w


# ----------------------------------------------------------------------------
# step 5: counter-based Gaussian noise [II-A]
# ----------------------------------------------------------------------------
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC'11).

    counter: uint32 [n, 4]; key: (k0, k1).  Each round multiplies words 0 and 2
    by the two Philox multipliers, and the new block is
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is advanced by the Weyl constants between rounds.
    """
    c = np.asarray(counter, dtype=np.uint64).reshape(-1, 4)
    m32 = np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + PHILOX_W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + PHILOX_W1) & 0xFFFFFFFF)
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & m32,
                          (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & m32)
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def box_muller(xa, xb):
    """Standard normal from two 32-bit words: u1 = (xa + 1) 2^-32 in (0, 1], u2 = xb 2^-32,
    z = sqrt(-2 ln u1) cos(2 pi u2).  |z| <= sqrt(64 ln 2) ~ 6.6604."""
    u1 = (np.asarray(xa, dtype=np.float64) + 1.0) * 2.0 ** -32
    u2 = np.asarray(xb, dtype=np.float64) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def beam_normals(seed: int, scan: int, inst: int, beams, word3=0):
    """(z_range, z_intensity) for beams, from Philox counter (beam, scan, inst, word3), key = seed
    (word3 = 0 for the single return; the echo index for multi-echo returns)."""
    beams = np.asarray(beams, dtype=np.uint64)
    ctr = np.zeros((len(beams), 4), dtype=np.uint64)
    ctr[:, 0] = beams
    ctr[:, 1] = scan
    ctr[:, 2] = inst
    ctr[:, 3] = word3
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    return box_muller(x[:, 0], x[:, 1]), box_muller(x[:, 2], x[:, 3])


# ----------------------------------------------------------------------------
# the whole path for one scan
# ----------------------------------------------------------------------------
def trace_limit(scene, sensor) -> float:
    """Largest first-hit distance that can still be detected: d_max plus the
    largest possible noise excursion (Box-Muller is bounded)."""
    if not sensor.noise_on:
        return float(sensor.d_max)
    return float(sensor.d_max) + BOX_MULLER_BOUND * float(np.max(scene.sigma_range))


def simulate(scene, sensor, pose, seed: int = 0, scan: int = 0, inst: int = 0, beams=None,
             rho=None, angle_exp=None, R=None, p=None):
    """Oracle for one scan.  Returns a dict of per-beam FP64/int arrays.

    beams: optional subset of beam indices (b = j * n_az + i); default all.
    rho: optional per-material R_lambda(0) used directly instead of the spectral
    table; angle_exp: optional per-material exponent k; R, p: optional rotation
    matrix / origin (FP64) overriding the pose.
    """
    with np.errstate(invalid="ignore", over="ignore"):
        return _simulate(scene, sensor, pose, seed, scan, inst, beams, rho, angle_exp, R, p)


def _rotate(R, s):
    """d = R s for every row of s; R is [3, 3] or one matrix per row [n, 3, 3].
    Each component is the plain three-term sum, left to right."""
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 2:
        R = R[None]
    return np.stack([R[:, r, 0] * s[:, 0] + R[:, r, 1] * s[:, 1] + R[:, r, 2] * s[:, 2] for r in range(3)], axis=1)


def _simulate(scene, sensor, pose, seed, scan, inst, beams, rho, angle_exp, R, p):
    n_all = sensor.n_beams
    beams = np.arange(n_all, dtype=np.int64) if beams is None else np.asarray(beams, dtype=np.int64)
    s_all = beam_directions(sensor).reshape(-1, 3)
    s = s_all[beams]
    Rm = rotation_from_quat(pose.q) if R is None else np.asarray(R, dtype=np.float64)
    o = np.asarray(pose.p, dtype=np.float64) if p is None else np.asarray(p, dtype=np.float64)
    return _trace_and_return(scene, sensor, beams, s, _rotate(Rm, s), o, seed, scan, inst, rho, angle_exp)


def _trace_and_return(scene, sensor, beams, s, d, o, seed, scan, inst, rho, angle_exp):
    """Steps 2-7 for beams with sensor-frame directions s, world directions d,
    origins o ([3] or [n, 3]) and Philox scan counter `scan` (scalar or per beam)."""
    # step 2: first hit within the traceable range (traced a little beyond it
    # so that hits straddling the limit are seen and can be flagged)
    t_lim = trace_limit(scene, sensor)
    fh = first_hit(scene, o, d, sensor.t_min, t_lim * (1 + 1e-5) + 1e-3)
    tri = fh["tri"]
    t1 = fh["t"]
    hit = (tri >= 0) & (t1 <= t_lim)
    safe = np.where(hit, tri, 0)

    # step 3 + 4: attributes of the hit triangle, return model
    n = face_normals(scene, safe)
    c = np.einsum("ij,ij->i", n, d)
    cos_t = np.abs(c)
    m = scene.material[safe].astype(np.int64)
    if rho is None:
        r0_tab, clamped = reflectance_at_wavelength(scene.spectra, sensor.wavelength_nm)
    else:
        r0_tab, clamped = np.asarray(rho, dtype=np.float64), False
    kexp = np.asarray(scene.angle_exp if angle_exp is None else angle_exp, dtype=np.float64)
    k_b = kexp[m]
    r_lambda = r0_tab[m] * np.where(k_b == 1.0, cos_t, cos_t ** k_b)

    # step 5: noise
    z_d, z_i = beam_normals(seed, scan, inst, beams)
    sig = scene.sigma_range.astype(np.float64)[m] if sensor.noise_on else np.zeros(len(beams))
    sig_i = float(sensor.sigma_intensity) if sensor.noise_on else 0.0
    d_n = t1 + sig * z_d

    # step 6: capability model
    r_l = (sensor.r_l_max / sensor.d_max) * d_n
    det = hit & (d_n > sensor.t_min) & (d_n <= sensor.d_max) & (r_l <= r_lambda)
    inten = np.maximum(0.0, r_lambda + sig_i * z_i)

    # step 7: outputs (misses and drops: valid 0, label all-ones, zeros elsewhere)
    out = dict(
        beams=beams,
        valid=det.astype(np.uint8),
        x=np.where(det, d_n * s[:, 0], 0.0),
        y=np.where(det, d_n * s[:, 1], 0.0),
        z=np.where(det, d_n * s[:, 2], 0.0),
        intensity=np.where(det, inten, 0.0),
        range=np.where(det, d_n, 0.0),
        label=np.where(det, scene.label[safe].astype(np.int64), MISS_LABEL).astype(np.uint32),
        tri=np.where(hit, tri, MISS_TRI).astype(np.uint32),
        t_hit=np.where(hit, t1, 0.0),
        material=np.where(hit, m, 0xFFFF).astype(np.uint16),
        normal=np.where(hit[:, None], n, 0.0),
        cos_theta=np.where(hit, cos_t, 0.0),
        r_lambda=np.where(hit, r_lambda, 0.0),
        hit=hit, wavelength_clamped=clamped, dir_world=d, dir_sensor=s,
    )
    # rays on which a 32-bit implementation may legitimately differ
    has = tri >= 0
    eps_e = EDGE_ABS_M + EDGE_REL * np.where(has, t1, 0.0)
    out["amb_tie"] = has & (fh["t_second"] - t1 < TIE_MARGIN_M)
    out["amb_edge"] = has & (fh["edge_in"] < eps_e)
    out["amb_near"] = np.where(has, fh["near_t"] <= t1 + TIE_MARGIN_M, np.isfinite(fh["near_t"]))
    out["amb_limit"] = has & (np.abs(t1 - t_lim) <= 1e-6 * (1.0 + t_lim))
    out["ambiguous"] = out["amb_tie"] | out["amb_edge"] | out["amb_near"] | out["amb_limit"]
    out["grazing"] = hit & (cos_t < 0.01)
    out["marginal"] = hit & ((np.abs(r_lambda - r_l) <= 1e-5 * r_lambda)
                             | (np.abs(d_n - sensor.d_max) <= 1e-5 * sensor.d_max)
                             | (np.abs(d_n - sensor.t_min) <= 1e-5))
    return out


def point_cloud(out, fields=("x", "y", "z", "intensity", "label", "range")):
    """Step 7 [Fig.1 caption]: the labelled point cloud lists the detected
    returns only; a miss or a dropped return has no point.  Points keep the
    beam order of the range image (b = j * n_az + i); `beam` gives each
    point's beam index (the dense index when `out` has no `beams` entry)."""
    valid = np.asarray(out["valid"]).reshape(-1)
    keep = np.flatnonzero(valid != 0)
    pc = {k: np.asarray(out[k]).reshape(-1)[keep] for k in fields}
    beams = np.asarray(out["beams"]) if "beams" in out else np.arange(len(valid))
    pc["beam"] = beams[keep]
    return pc


# ----------------------------------------------------------------------------
# beam divergence and multi-echo returns [IV, named there as future work]
# ----------------------------------------------------------------------------
# The paper's conclusion names beam divergence and multi-echo LiDAR as the next
# physical effects to model, without a model.  Reading used here:
#  * a beam is a cone of full angle delta around its axis s, sampled by K
#    sub-rays of equal power 1/K: sub-ray 0 is the axis, sub-ray k >= 1 is the
#    axis turned by r_k = (delta / 2) sqrt(k / (K - 1)) towards the direction
#    cos(b_k) e_theta + sin(b_k) e_phi, b_k = k * pi (3 - sqrt 5) (a Vogel
#    spiral over the cone's disk), with e_theta, e_phi the unit azimuth and
#    elevation tangents at s;
#  * every sub-ray gets its first hit and its noise-free R_lambda (eq.4);
#  * the hits, ordered by (t, k), form echoes: a gap larger than the range
#    resolution starts a new echo;
#  * an echo's strength is P = (1/K) sum R_lambda,k over its sub-rays (the
#    returned power fraction), its range the R_lambda-weighted mean
#    t = t_first + sum R_k (t_k - t_first) / sum R_k (plain mean if all R are
#    0), its label and material those of its strongest sub-ray (smallest k on
#    ties);
#  * echo e gets range noise and intensity noise from Philox counter
#    (beam, scan, instance, e) and the eq.5 test with P in place of R_lambda;
#  * the first E echoes in range order are reported.
# With K = 1 and delta = 0, echo 0 is exactly the single return of simulate().

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def subray_pattern(n_sub: int, divergence_rad: float):
    """(r_k, b_k) for k = 0..K-1: angle from the beam axis and direction around it."""
    k = np.arange(n_sub, dtype=np.float64)
    r = np.zeros(n_sub) if n_sub == 1 else (0.5 * float(divergence_rad)) * np.sqrt(k / (n_sub - 1))
    return r, k * GOLDEN_ANGLE


def subray_directions(sensor, beams, n_sub: int, divergence_rad: float) -> np.ndarray:
    """Sensor-frame unit directions [n_beams, K, 3] of the sub-rays of the given beams."""
    theta, phi = beam_angles(sensor)
    beams = np.asarray(beams, dtype=np.int64)
    th = theta[beams % sensor.n_az][:, None]
    ph = phi[beams // sensor.n_az][:, None]
    ct, st, cp, sp = np.cos(th), np.sin(th), np.cos(ph), np.sin(ph)
    axis = np.stack([cp * ct, cp * st, sp * np.ones_like(ct)], axis=-1)          # [n, 1, 3]
    e_th = np.stack([-st, ct, np.zeros_like(ct)], axis=-1)
    e_ph = np.stack([-sp * ct, -sp * st, cp], axis=-1)
    r, b = subray_pattern(n_sub, divergence_rad)
    r, b = r[None, :, None], b[None, :, None]
    return np.cos(r) * axis + np.sin(r) * (np.cos(b) * e_th + np.sin(b) * e_ph)


def simulate_echoes(scene, sensor, pose, n_sub: int, max_echoes: int, divergence_rad: float, echo_sep_m: float,
                    seed: int = 0, scan: int = 0, inst: int = 0, beams=None):
    """Oracle for one scan with divergent beams and multi-echo returns.

    Returns per-echo arrays [E, n] (valid, range, intensity, label, x, y, z,
    tri, t_hit, material, r_lambda (= P)), ``n_echoes`` [n] (echoes formed),
    the per-sub-ray hits, and ``ambiguous`` [n] (a sub-ray is ambiguous in
    the sense of simulate(), or two of its hits straddle the echo separation
    or the ordering within 1e-6 m) and ``marginal`` [E, n].
    """
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        return _simulate_echoes(scene, sensor, pose, n_sub, max_echoes, divergence_rad, echo_sep_m, seed, scan,
                                inst, beams)


def _simulate_echoes(scene, sensor, pose, n_sub, max_echoes, divergence_rad, echo_sep_m, seed, scan, inst, beams):
    n_all = sensor.n_beams
    beams = np.arange(n_all, dtype=np.int64) if beams is None else np.asarray(beams, dtype=np.int64)
    n, K, E = len(beams), int(n_sub), int(max_echoes)
    sdir = subray_directions(sensor, beams, K, divergence_rad).reshape(-1, 3)
    R = rotation_from_quat(pose.q)
    o = np.asarray(pose.p, dtype=np.float64)
    d = _rotate(R, sdir)
    t_lim = trace_limit(scene, sensor)
    fh = first_hit(scene, o, d, sensor.t_min, t_lim * (1 + 1e-5) + 1e-3)
    tri = fh["tri"]
    t1 = fh["t"]
    hit = (tri >= 0) & (t1 <= t_lim)
    safe = np.where(hit, tri, 0)
    nrm = face_normals(scene, safe)
    cos_t = np.abs(np.einsum("ij,ij->i", nrm, d))
    m = scene.material[safe].astype(np.int64)
    r0_tab, clamped = reflectance_at_wavelength(scene.spectra, sensor.wavelength_nm)
    kexp = np.asarray(scene.angle_exp, dtype=np.float64)[m]
    r_l = r0_tab[m] * np.where(kexp == 1.0, cos_t, cos_t ** kexp)
    has = tri >= 0
    eps_e = EDGE_ABS_M + EDGE_REL * np.where(has, t1, 0.0)
    amb_sub = ((has & (fh["t_second"] - t1 < TIE_MARGIN_M)) | (has & (fh["edge_in"] < eps_e))
               | np.where(has, fh["near_t"] <= t1 + TIE_MARGIN_M, np.isfinite(fh["near_t"]))
               | (has & (np.abs(t1 - t_lim) <= 1e-6 * (1.0 + t_lim))))
    shape = (n, K)
    hit, t1, tri, r_l, m, amb_sub, cos_t = (a.reshape(shape) for a in (hit, t1, tri, r_l, m, amb_sub, cos_t))
    label = scene.label[np.where(hit, tri, 0)].astype(np.int64)

    out = {k: np.zeros((E, n)) for k in ("range", "intensity", "x", "y", "z", "t_hit", "r_lambda")}
    out["valid"] = np.zeros((E, n), np.uint8)
    out["label"] = np.full((E, n), MISS_LABEL, np.uint32)
    out["tri"] = np.full((E, n), MISS_TRI, np.uint32)
    out["material"] = np.full((E, n), 0xFFFF, np.uint16)
    out["marginal"] = np.zeros((E, n), bool)
    out["grazing"] = np.zeros((E, n), bool)
    out["amb_dom"] = np.zeros((E, n), bool)
    n_echo = np.zeros(n, np.int64)
    ambiguous = amb_sub.any(axis=1)
    sig_all = scene.sigma_range.astype(np.float64)
    axis = sdir.reshape(n, K, 3)[:, 0, :]
    zs = [beam_normals(seed, scan, inst, beams, word3=e) for e in range(E)]
    for b in range(n):
        ks = [k for k in range(K) if hit[b, k]]
        ks.sort(key=lambda k: (t1[b, k], k))
        groups = []
        for idx, k in enumerate(ks):
            if idx == 0 or t1[b, k] - t1[b, ks[idx - 1]] > echo_sep_m:
                groups.append([k])
            else:
                groups.append(groups.pop() + [k])
            if idx > 0:
                # a 32-bit range is good to about 1e-6 relative: gaps that close to the separation
                # (or to zero, where the order decides the first range) may group differently
                gap = t1[b, k] - t1[b, ks[idx - 1]]
                if abs(gap - echo_sep_m) <= 1e-5 * (1.0 + t1[b, k]) or gap <= TIE_MARGIN_M:
                    ambiguous[b] = True
        n_echo[b] = len(groups)
        for e, g in enumerate(groups[:E]):
            rs = np.array([r_l[b, k] for k in g])
            ts = np.array([t1[b, k] for k in g])
            P = rs.sum() / K
            t0 = ts[0]
            te = t0 + (np.sum(rs * (ts - t0)) / rs.sum() if rs.sum() > 0 else np.mean(ts - t0))
            order = np.argsort(-rs, kind="stable")
            dom = min(g[q] for q in range(len(g)) if rs[q] == rs.max())     # strongest, smallest k on ties
            # strongest sub-ray decided within 32-bit rounding: another one within 1e-5 relative
            if len(g) > 1 and rs[order[1]] >= rs[order[0]] * (1.0 - 1e-5):
                out["amb_dom"][e, b] = True
            mm = int(m[b, dom])
            z_d, z_i = zs[e][0][b], zs[e][1][b]
            sig = sig_all[mm] if sensor.noise_on else 0.0
            sig_i = float(sensor.sigma_intensity) if sensor.noise_on else 0.0
            dn = te + sig * z_d
            rlim = (sensor.r_l_max / sensor.d_max) * dn
            det = (dn > sensor.t_min) and (dn <= sensor.d_max) and (rlim <= P)
            out["t_hit"][e, b] = te
            out["r_lambda"][e, b] = P
            out["tri"][e, b] = tri[b, dom]
            out["material"][e, b] = mm
            out["marginal"][e, b] = ((abs(P - rlim) <= 1e-5 * max(P, 1e-30)) or abs(dn - sensor.d_max) <= 1e-5 * sensor.d_max
                                     or abs(dn - sensor.t_min) <= 1e-5)
            out["grazing"][e, b] = bool(np.any(np.array([cos_t[b, k] for k in g]) < 0.01))
            if det:
                out["valid"][e, b] = 1
                out["range"][e, b] = dn
                out["intensity"][e, b] = max(0.0, P + sig_i * z_i)
                out["label"][e, b] = label[b, dom]
                out["x"][e, b], out["y"][e, b], out["z"][e, b] = dn * axis[b]
    out.update(beams=beams, n_echoes=n_echo, ambiguous=ambiguous, wavelength_clamped=clamped,
               sub_hit=hit, sub_t=t1, sub_tri=tri, sub_r_lambda=r_l, sub_dir_sensor=sdir.reshape(n, K, 3))
    return out


# ----------------------------------------------------------------------------
# partial sweep per simulation tick, rolling-shutter pose [II-A]
# ----------------------------------------------------------------------------
# Section II-A renders, at every engine tick, only the part of FOV_h that the
# spinning head has covered since the previous tick (from the spin rate omega_l
# and the tick length dt).  Here every column fired during the tick is traced
# with the pose the sensor has at the moment that column fires: the pose moves
# linearly in position and along the great arc (slerp) in orientation from the
# pose at the tick start to the pose at the tick end.  With equal start and end
# poses this is the paper's one-pose-per-tick model.

SLERP_LINEAR_BELOW = 1e-6      # arc angle (rad) under which the interpolation is linear


def sweep_window(head_deg_begin, spin_hz, dt_s):
    """Head-angle interval [a, b) swept during one tick: b = a + 360 omega_l dt
    (degrees, unwrapped: revolution s covers [360 s, 360 (s + 1)) + az0)."""
    a = float(head_deg_begin)
    return a, a + 360.0 * float(spin_hz) * float(dt_s)


def column_coordinate(sensor, x, s):
    """c_s(x) = ((x - az0) - 360 s) N_az / FOV_h: head angle x in units of
    azimuth steps of revolution s, evaluated in exactly this order in FP64."""
    return ((float(x) - sensor.az0_deg) - 360.0 * s) * sensor.n_az / sensor.fov_h_deg


def sweep_columns(sensor, a, b):
    """Columns fired while the head turns over [a, b) (degrees, b - a <= 360).

    Column i of revolution (scan) s >= 0 points at head angle
    A = 360 s + az0 + i FOV_h / N_az; it is fired iff a <= A < b, decided in
    column coordinates as ceil(c_s(a)) <= i < ceil(c_s(b)).  A window of at
    most one revolution can only reach revolutions s_a = floor((a - az0) / 360)
    and s_a + 1.  Returns the non-empty runs [(s, i_begin, i_end), ...] in
    firing order.
    """
    if not (b >= a and b - a <= 360.0):
        raise ValueError("a tick sweeps between 0 and 360 degrees")
    s_a = math.floor((float(a) - sensor.az0_deg) / 360.0)
    runs = []
    for s in (s_a, s_a + 1):
        if s < 0:
            continue
        lo = max(0, math.ceil(column_coordinate(sensor, a, s)))
        hi = min(sensor.n_az, math.ceil(column_coordinate(sensor, b, s)))
        if hi > lo:
            runs.append((int(s), int(lo), int(hi)))
    return runs


def column_time_fraction(sensor, s, i, a, b):
    """tau = (A - a) / (b - a): the fraction of the tick at which column (s, i) fires,
    with A = 360 s + (az0 + i FOV_h / N_az)."""
    A = 360.0 * s + (sensor.az0_deg + i * (sensor.fov_h_deg / sensor.n_az))
    return (A - a) / (b - a)


def slerp(qa, qb, tau):
    """Quaternion on the great arc from qa to qb at fraction tau (Shoemake, SIGGRAPH 1985).

    qb is negated when qa . qb < 0, so that the shorter of the two arcs between
    the rotations is taken.  With unit ends ua, ub and arc angle W = acos(ua . ub):
    q = sin((1 - tau) W) / sin W ua + sin(tau W) / sin W ub.  Below
    SLERP_LINEAR_BELOW the arc is replaced by the chord qa + tau (qb - qa)
    between the given quaternions (not renormalised: rotation_from_quat
    normalises), so equal ends give back exactly the given quaternion.
    """
    qa = np.asarray(qa, dtype=np.float64)
    qb = np.asarray(qb, dtype=np.float64)
    ua = qa / np.linalg.norm(qa)
    ub = qb / np.linalg.norm(qb)
    dot = float(np.dot(ua, ub))
    if dot < 0.0:
        qb, ub, dot = -qb, -ub, -dot
    w = math.acos(min(dot, 1.0))
    if w < SLERP_LINEAR_BELOW:
        return qa + tau * (qb - qa)
    sw = math.sin(w)
    return (math.sin((1.0 - tau) * w) / sw) * ua + (math.sin(tau * w) / sw) * ub


def sweep_pose(pose_a, pose_b, tau):
    """(R, p) at fraction tau of the tick: p = pa + tau (pb - pa), R from slerp."""
    pa = np.asarray(pose_a.p, dtype=np.float64)
    pb = np.asarray(pose_b.p, dtype=np.float64)
    return rotation_from_quat(slerp(pose_a.q, pose_b.q, tau)), pa + tau * (pb - pa)


def simulate_sweep(scene, sensor, pose_a, pose_b, head_deg_begin, spin_hz, dt_s, seed: int = 0,
                   inst: int = 0, beams=None):
    """Oracle for one tick of a spinning sensor.

    The columns fired during the tick (``sweep_columns``) are traced with the
    pose of their firing time; the Philox counter of beam (j, i) of revolution
    s is (j N_az + i, s, inst, 0), so the ticks of one revolution together
    reproduce ``simulate(..., scan=s)`` when the pose does not change.
    beams: optional subset of range-image slots b = j N_az + i, which must lie
    in fired columns.  Returns the ``simulate`` dict plus ``runs``, ``scan``
    (per beam) and ``tau`` (per beam).
    """
    a, b = sweep_window(head_deg_begin, spin_hz, dt_s)
    runs = sweep_columns(sensor, a, b)
    col_scan = np.full(sensor.n_az, -1, dtype=np.int64)
    for s_, lo, hi in runs:
        col_scan[lo:hi] = s_
    fired = np.flatnonzero(col_scan >= 0)
    if beams is None:
        beams = (np.arange(sensor.n_ch, dtype=np.int64)[:, None] * sensor.n_az + fired[None, :]).reshape(-1)
        beams = np.sort(beams)
    beams = np.asarray(beams, dtype=np.int64)
    col = beams % sensor.n_az
    if np.any(col_scan[col] < 0):
        raise ValueError("beam outside the columns fired in this tick")
    scan_b = col_scan[col]
    tau_c = {int(i): column_time_fraction(sensor, int(col_scan[i]), int(i), a, b) for i in np.unique(col)}
    poses = {i: sweep_pose(pose_a, pose_b, t) for i, t in tau_c.items()}
    Rb = np.stack([poses[int(i)][0] for i in col]) if len(col) else np.zeros((0, 3, 3))
    ob = np.stack([poses[int(i)][1] for i in col]) if len(col) else np.zeros((0, 3))
    s = beam_directions(sensor).reshape(-1, 3)[beams]
    with np.errstate(invalid="ignore", over="ignore"):
        out = _trace_and_return(scene, sensor, beams, s, _rotate(Rb, s), ob, seed, scan_b, inst, None, None)
    out["runs"] = runs
    out["scan"] = scan_b
    out["tau"] = np.array([tau_c[int(i)] for i in col], dtype=np.float64)
    return out


# ----------------------------------------------------------------------------
# dynamic scenes: meshes placed in the world by moving actors [II-B]
# ----------------------------------------------------------------------------
# An actor places a mesh (object-space triangles with per-triangle materials)
# in the world with a rigid transform x_world = R(q) x_object + p and gives all
# of its triangles one instance label (Section II-B labels every object
# instance).  The first hit is taken over one triangle soup: the static
# triangles first, then every actor's triangles in actor order, with FP64
# world vertices, so ties are broken by that order.

def actor_vertices(mesh, actor) -> np.ndarray:
    """World vertices R(q) v + p (FP64) of the mesh placed by the actor."""
    R = rotation_from_quat(actor.q)
    v = np.asarray(mesh.vertices, dtype=np.float64)
    return v @ R.T + np.asarray(actor.p, dtype=np.float64)


def scene_with_actors(scene, meshes, actors, mesh_vertices=None):
    """The static scene and the placed actors as one soup (FP64 vertices).

    mesh_vertices: optional per-mesh replacement vertex arrays (deformed meshes,
    same topology).  Returns (soup, tri_base) with tri_base[a] the index of
    actor a's first triangle in the soup.
    """
    from dataclasses import replace
    verts = [np.asarray(scene.vertices, dtype=np.float64)]
    idx = [np.asarray(scene.indices, dtype=np.int64)]
    mat = [np.asarray(scene.material)]
    lab = [np.asarray(scene.label)]
    nv, nt = len(verts[0]), scene.n_tri
    tri_base = []
    for a in actors:
        m = meshes[a.mesh]
        mv = m if mesh_vertices is None or mesh_vertices[a.mesh] is None else replace(m, vertices=mesh_vertices[a.mesh])
        verts.append(actor_vertices(mv, a))
        idx.append(np.asarray(m.indices, dtype=np.int64) + nv)
        mat.append(np.asarray(m.material))
        lab.append(np.full(m.n_tri, a.label, dtype=np.uint32))
        tri_base.append(nt)
        nv += len(m.vertices)
        nt += m.n_tri
    soup = replace(scene, vertices=np.concatenate(verts), indices=np.concatenate(idx).astype(np.uint32),
                   material=np.concatenate(mat).astype(np.uint16), label=np.concatenate(lab).astype(np.uint32))
    return soup, np.array(tri_base, dtype=np.int64)


def simulate_actors(scene, meshes, actors, sensor, pose, seed: int = 0, scan: int = 0, beams=None,
                    mesh_vertices=None):
    """Oracle for one scan of a dynamic scene; the ``simulate`` dict plus ``tri_base``."""
    soup, tri_base = scene_with_actors(scene, meshes, actors, mesh_vertices)
    out = simulate(soup, sensor, pose, seed=seed, scan=scan, beams=beams)
    out["tri_base"] = tri_base
    return out


# ----------------------------------------------------------------------------
# adjoint: gradients of an intensity/depth loss with the hit triangles fixed
# ----------------------------------------------------------------------------
def _fixed_triangle_forward(scene, s, tri, R, p, rho, kexp, sig_i=0.0, z_i=None):
    """I and t for beams whose hit triangle is held fixed.

    c = n . d with d = R s; t = n . (v0 - p) / c (ray/plane distance of the
    fixed triangle); R_lambda = rho_m |c|^k_m (eq.4 with the cos^k reading).
    The intensity is R_lambda itself, or, with intensity noise (sig_i > 0 and
    the per-beam standard normals z_i of the forward scan), the forward's
    max(0, R_lambda + sig_i z_i).  Also returns the mask of beams whose
    intensity is not clamped at 0 (the ones through which R_lambda reaches I).
    """
    v = scene.vertices.astype(np.float64)[scene.indices[tri].astype(np.int64)]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    d = s @ R.T
    c = np.einsum("ij,ij->i", n, d)
    t = np.einsum("ij,ij->i", n, v[:, 0] - p) / c
    m = scene.material[tri].astype(np.int64)
    r_lam = rho[m] * np.abs(c) ** kexp[m]
    if z_i is None or sig_i == 0.0:
        return r_lam, t, n, d, c, m, np.ones(len(t), dtype=bool)
    pre = r_lam + sig_i * np.asarray(z_i, dtype=np.float64)
    return np.maximum(0.0, pre), t, n, d, c, m, pre > 0.0


def calib_loss(scene, sensor, pose_ref, tri, beams, rho, kexp, dp, dw, I_tgt, t_tgt, lam_d=1.0, sig_i=0.0,
               z_i=None):
    """L = mean((I - I*)^2) + lam_d * mean((t - t*)^2) over the given beams.

    Pose: p = p_ref + dp, R = Exp(dw) R_ref.  I as in ``_fixed_triangle_forward``
    (with intensity noise when sig_i and z_i are given).  FP64.
    """
    s = beam_directions(sensor).reshape(-1, 3)[np.asarray(beams)]
    R = so3_exp(dw) @ rotation_from_quat(pose_ref.q)
    p = np.asarray(pose_ref.p, dtype=np.float64) + np.asarray(dp, dtype=np.float64)
    I, t, *_ = _fixed_triangle_forward(scene, s, np.asarray(tri), R, p,
                                       np.asarray(rho, np.float64), np.asarray(kexp, np.float64), sig_i, z_i)
    N = len(beams)
    return float(np.sum((I - I_tgt) ** 2) / N + lam_d * np.sum((t - t_tgt) ** 2) / N)


def calib_grad(scene, sensor, pose_ref, tri, beams, rho, kexp, dp, dw, I_tgt, t_tgt, lam_d=1.0, sig_i=0.0,
               z_i=None):
    """Analytic gradient of ``calib_loss``: returns (d_rho[nmat], d_k[nmat], d_pose6[6]).

    With g_I = dL/dI and g_t = dL/dt per beam, and g_I taken as 0 where the
    intensity is clamped at 0 (I = max(0, R_lambda + sig_i z_i) does not move
    with R_lambda there):
      dL/drho_m = sum g_I |c|^k;  dL/dk_m = sum g_I rho |c|^k ln|c|;
      dL/dp = sum -g_t n / c;
      dL/d(left rotation perturbation) = sum gamma (d x n),
        gamma = g_I rho k |c|^(k-1) sgn(c) - g_t t / c,
      mapped to dw through the left Jacobian of Exp at dw.
    """
    rho = np.asarray(rho, np.float64)
    kexp = np.asarray(kexp, np.float64)
    s = beam_directions(sensor).reshape(-1, 3)[np.asarray(beams)]
    R = so3_exp(dw) @ rotation_from_quat(pose_ref.q)
    p = np.asarray(pose_ref.p, dtype=np.float64) + np.asarray(dp, dtype=np.float64)
    I, t, n, d, c, m, live = _fixed_triangle_forward(scene, s, np.asarray(tri), R, p, rho, kexp, sig_i, z_i)
    N = len(beams)
    gI = np.where(live, 2.0 * (I - I_tgt) / N, 0.0)
    gt = 2.0 * lam_d * (t - t_tgt) / N
    ac = np.abs(c)
    k_b = kexp[m]
    nmat = len(rho)
    d_rho = np.bincount(m, weights=gI * ac ** k_b, minlength=nmat)
    d_k = np.bincount(m, weights=gI * rho[m] * ac ** k_b * np.log(ac), minlength=nmat)
    d_p = np.sum((-gt / c)[:, None] * n, axis=0)
    gamma = gI * rho[m] * k_b * ac ** (k_b - 1.0) * np.sign(c) - gt * t / c
    d_left = np.sum(gamma[:, None] * np.cross(d, n), axis=0)
    d_w = so3_left_jacobian(dw).T @ d_left
    return d_rho, d_k, np.concatenate([d_p, d_w])


def calib_grad_spectral(scene, sensor, pose_ref, tri, beams, spectra, kexp, dp, dw, I_tgt, t_tgt, lam_d=1.0,
                        sig_i=0.0, z_i=None):
    """Gradient of ``calib_loss`` with R_lambda(0) taken from the spectral table
    at the sensor wavelength: returns (d_spectra[nmat, nbins], d_k, d_pose6).

    R_lambda(0)_m = sum_b w_b T[m, b] with the interpolation weights w of the
    sensor wavelength, so dL/dT[m, b] = w_b dL/dR_lambda(0)_m: only the one or
    two bins around the wavelength receive gradient.
    """
    T = np.asarray(spectra, np.float64)
    rho = reflectance_at_wavelength(T, sensor.wavelength_nm)[0]
    d_rho, d_k, d_pose = calib_grad(scene, sensor, pose_ref, tri, beams, rho, kexp, dp, dw, I_tgt, t_tgt, lam_d,
                                    sig_i, z_i)
    w = spectral_weights(T.shape[1], sensor.wavelength_nm)
    return np.outer(d_rho, w), d_k, d_pose
