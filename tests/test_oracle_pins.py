"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed
form, a published known-answer vector, an invariance, a special case that
reduces to a textbook formula, or an independent brute force written with a
different algorithm.  A plausible mistake in the oracle (dropped term, sign,
transposed operand, wrong index, wrong comparator) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scene(verts, tris, mats=None, labels=None, spectra=None, nmat=1, sigma=0.0, kexp=None):
    verts = np.asarray(verts, np.float32)
    tris = np.asarray(tris, np.uint32)
    nt = len(tris)
    mats = np.zeros(nt, np.uint16) if mats is None else np.asarray(mats, np.uint16)
    labels = np.arange(1, nt + 1, dtype=np.uint32) if labels is None else np.asarray(labels, np.uint32)
    if spectra is None:
        spectra = np.full((nmat, 61), 0.5, np.float32)
    return S.Scene(verts, tris, mats, labels, np.asarray(spectra, np.float32),
                   np.full(len(spectra), sigma, np.float32),
                   np.ones(len(spectra), np.float32) if kexp is None else np.asarray(kexp, np.float32))


def _ground(half=1000.0, z=0.0, **kw):
    v = [[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]]
    return _scene(v, [[0, 1, 2], [0, 2, 3]], **kw)


# ----------------------------------------------------------------------------
# Philox / Box-Muller (noise model, Section II-A)
# ----------------------------------------------------------------------------
def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for vec in kat["vectors"]:
        ctr = np.array([[int(x, 16) for x in vec["counter"]]], np.uint32)
        key = tuple(int(x, 16) for x in vec["key"])
        out = O.philox4x32_10(ctr, key)[0]
        assert [f"{int(x):08x}" for x in out] == vec["out"]


def test_box_muller_bound_and_moments():
    # extreme inputs: u1 = 2^-32 gives the largest |z| = sqrt(64 ln 2)
    zmax = O.box_muller(np.uint32(0), np.uint32(0))
    assert abs(float(zmax) - math.sqrt(64 * math.log(2))) < 1e-12
    assert abs(float(zmax)) <= O.BOX_MULLER_BOUND
    assert float(O.box_muller(np.uint32(0xFFFFFFFF), np.uint32(123))) == 0.0   # u1 = 1
    zd, zi = O.beam_normals(seed=12345, scan=3, inst=1, beams=np.arange(1_000_000))
    for z in (zd, zi):
        assert np.all(np.abs(z) <= O.BOX_MULLER_BOUND)
        assert abs(z.mean()) < 5e-3
        assert abs(z.var() - 1.0) < 5e-3
        assert abs(np.mean(z ** 3)) < 1e-2         # symmetric
        assert abs(np.mean(z ** 4) - 3.0) < 3e-2   # Gaussian kurtosis
    assert abs(np.corrcoef(zd, zi)[0, 1]) < 5e-3


# ----------------------------------------------------------------------------
# eq.1-3 beam convention (P6)
# ----------------------------------------------------------------------------
def test_beam_convention_matches_pinhole_eq3():
    """Projecting the oracle's beam direction with K_c (eq.1-2) gives the corrected eq.3."""
    W, fov_c = 1024.0, math.radians(90.0)
    f = W / (2 * math.tan(fov_c / 2))
    K = np.array([[f, 0, W / 2], [0, f, W / 2], [0, 0, 1.0]])
    sensor = S.Sensor(np.array([-20.0, -7.5, 0.0, 3.3, 30.0]), 360)
    s = O.beam_directions(sensor)
    theta, phi = O.beam_angles(sensor)
    for j in range(len(phi)):
        for i in list(range(0, 40, 7)) + list(range(330, 360, 6)):   # |theta| < 45 deg
            th = theta[i] if theta[i] < math.pi else theta[i] - 2 * math.pi
            x, y, z = s[j, i]
            cam = np.array([y, -z, x])          # camera looks along the sensor x axis
            uvw = K @ cam
            nx, ny = O.pixel_of_beam(th, phi[j], W, fov_c)
            assert abs(uvw[0] / uvw[2] - nx) < 1e-9
            assert abs(uvw[1] / uvw[2] - ny) < 1e-9
    assert np.allclose(np.linalg.norm(s, axis=-1), 1.0, atol=1e-15)
    # azimuth 0 is +x, azimuth 90 deg is +y, positive elevation is +z
    s4 = O.beam_directions(S.Sensor(np.array([0.0, 90.0]), 4))
    assert np.allclose(s4[0, 0], [1, 0, 0]) and np.allclose(s4[0, 1], [0, 1, 0], atol=1e-15)
    assert np.allclose(s4[1, 0], [0, 0, 1], atol=1e-15)


def test_quaternion_rotation_matches_rodrigues():
    rng = np.random.default_rng(0)
    for _ in range(20):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(-3, 3)
        q = np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis]
        R = O.rotation_from_quat(q * 3.0)          # scale must not matter
        assert np.allclose(R, O.so3_exp(ang * axis), atol=1e-12)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12


# ----------------------------------------------------------------------------
# P1: ray to a plane at known distance and angle (eq.4, eq.5)
# ----------------------------------------------------------------------------
def test_ground_plane_closed_form_16ch_numbers():
    """Ground seen from h = 1.5 m: t = h / sin|phi|, cos(theta_inc) = sin|phi|, I = rho cos."""
    h, rho = 1.5, 0.5
    scene = _ground(spectra=np.full((1, 61), rho, np.float32))
    sensor = S.Sensor(np.array([-15.0, -7.0, -8.0, -9.0]), 8, d_max=100.0, r_l_max=0.8, noise_on=False)
    pose = S.Pose(np.array([0, 0, h], np.float32), np.array([1, 0, 0, 0], np.float32))
    r = O.simulate(scene, sensor, pose)
    n_az = sensor.n_az
    for j, phi_deg in enumerate(sensor.elev_deg):
        sp = math.sin(math.radians(abs(phi_deg)))
        b = j * n_az + 3
        assert abs(r["t_hit"][b] - h / sp) < 1e-12 * (h / sp)
        assert abs(r["cos_theta"][b] - sp) < 1e-12
        assert abs(r["r_lambda"][b] - rho * sp) < 1e-12
        # capability model: detected iff 0.8/100 * d <= rho sin|phi|, i.e. sin^2|phi| >= 0.8 h /(100 rho)
        expect = (0.8 / 100.0) * (h / sp) <= rho * sp
        assert bool(r["valid"][b]) == expect
    # the numbers quoted for the 16-channel configuration
    b15 = 0 * n_az
    assert abs(r["t_hit"][b15] - 5.79555) < 5e-6
    assert abs(r["cos_theta"][b15] - 0.258819) < 5e-7
    assert abs(r["intensity"][b15] - 0.129410) < 5e-7
    assert abs(0.8 / 100 * r["range"][b15] - 0.046364) < 5e-7
    assert r["valid"][b15] == 1
    b7 = 1 * n_az
    assert abs(r["t_hit"][b7] - 12.3083) < 5e-5 and r["valid"][b7] == 0
    # cutoff elevation: sin^2|phi| = 0.8 * 1.5 / (100 * 0.5) -> |phi| = 8.91 deg
    cut = math.degrees(math.asin(math.sqrt(0.8 * 1.5 / 50.0)))
    assert abs(cut - 8.91) < 5e-3
    assert r["valid"][3 * n_az] == 1 and r["valid"][2 * n_az] == 0     # -9 kept, -8 dropped


def test_point_cloud_of_ground_plane_closed_form():
    """Point cloud over a ground plane: exactly the channels below the eq.5 cutoff elevation
    (sin^2|phi| >= R_L,max h / (d_max rho), |phi| >= 8.91 deg here) give points, every azimuth
    of them, in beam order, each at range h / sin|phi| with z = -h in the sensor frame."""
    h, rho = 1.5, 0.5
    scene = _ground(spectra=np.full((1, 61), rho, np.float32))
    elev = np.array([-15.0, 10.0, -7.0, -9.0, -8.0, -11.0, 0.0])
    sensor = S.Sensor(elev, 12, d_max=100.0, r_l_max=0.8, noise_on=False)
    pose = S.Pose(np.array([0, 0, h], np.float32), np.array([1, 0, 0, 0], np.float32))
    pc = O.point_cloud(O.simulate(scene, sensor, pose))
    cut = math.asin(math.sqrt(0.8 * h / (100.0 * rho)))
    kept = [j for j, e in enumerate(elev) if e < 0 and math.radians(-e) >= cut]
    assert kept == [0, 3, 5]
    expect_beams = np.array([j * 12 + i for j in kept for i in range(12)])
    np.testing.assert_array_equal(pc["beam"], expect_beams)
    phi = np.radians(-elev[expect_beams // 12])
    np.testing.assert_allclose(pc["range"], h / np.sin(phi), rtol=1e-12)
    np.testing.assert_allclose(pc["z"], -h, rtol=1e-12)
    np.testing.assert_allclose(np.hypot(pc["x"], pc["y"]), h / np.tan(phi), rtol=1e-12)
    # triangle 0 (label 1) is the half y < x of the square, triangle 1 (label 2) the half y > x
    np.testing.assert_array_equal(pc["label"], np.where(pc["y"] < pc["x"], 1, 2))


def test_tilted_plane_distance_and_angle():
    """Plane n.x = h at arbitrary orientation: t = (h - n.o)/(n.d), cos = |n.d|, I = rho cos^k."""
    rng = np.random.default_rng(5)
    for trial in range(10):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        hgt = rng.uniform(5, 40)
        # big square in the plane
        u = np.cross(n, [0.3, 0.5, 0.8])
        u /= np.linalg.norm(u)
        w = np.cross(n, u)
        c0 = n * hgt
        L = 2000.0
        v = [c0 + L * (a * u + b * w) for a, b in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
        kexp = rng.uniform(0.5, 2.5)
        scene = _scene(v, [[0, 1, 2], [0, 2, 3]], spectra=np.full((1, 61), 0.7, np.float32), kexp=[kexp])
        sensor = S.Sensor(np.linspace(-30, 30, 7), 12, d_max=999.0, noise_on=False)
        pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
        r = O.simulate(scene, sensor, pose)
        d = r["dir_world"]
        nd = d @ n
        # float32 vertices move the plane by at most ~1e-4 m; compare loosely there
        t_expect = hgt / nd
        hit = (t_expect > 0) & (t_expect <= 999.0)
        assert np.array_equal(r["hit"], hit)
        assert np.allclose(r["t_hit"][hit], t_expect[hit], rtol=1e-5)
        assert np.allclose(r["cos_theta"][hit], np.abs(nd[hit]), atol=1e-6)
        assert np.allclose(r["r_lambda"][hit], 0.7 * np.abs(nd[hit]) ** kexp, rtol=1e-5)


# ----------------------------------------------------------------------------
# P2: ray to a sphere
# ----------------------------------------------------------------------------
def test_sphere_facet_centroid_exact():
    """A ray from outside through the centre and a facet centroid hits that facet at
    t = |o - C| - |c_f - C|."""
    C = np.array([3.0, -2.0, 1.0])
    v, tris = S.uv_sphere(C, 2.0, 16, 9)
    scene = _scene(v, tris)
    vv = scene.vertices.astype(np.float64)
    rng = np.random.default_rng(1)
    for k in rng.choice(len(tris), 30, replace=False):
        cf = vv[scene.indices[k]].mean(axis=0)
        u = (cf - C) / np.linalg.norm(cf - C)
        dist = rng.uniform(5, 50)
        o = C + dist * u
        # keep the ray off the facet's edges: the centroid is well inside it
        fh = O.first_hit(scene, o[None], -u[None], 0.01, 1e3)
        assert fh["tri"][0] == k
        assert abs(fh["t"][0] - (dist - np.linalg.norm(cf - C))) < 1e-9


def test_fine_sphere_within_sag_bound():
    """256 x 128 UV sphere: t within r (1 - cos(pi/128)) / cos(incidence) of the analytic sphere."""
    C = np.array([0.0, 0.0, 0.0])
    r = 3.0
    v, tris = S.uv_sphere(C, r, 256, 128)
    scene = _scene(v, tris)
    rng = np.random.default_rng(2)
    o = np.array([12.0, 1.0, 0.5])
    dirs = (C - o) + rng.uniform(-2.0, 2.0, size=(200, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    fh = O.first_hit(scene, o[None], dirs, 0.01, 100.0)
    b = dirs @ (C - o)
    disc = b * b - (np.dot(C - o, C - o) - r * r)
    hit = disc > 0
    t_an = b - np.sqrt(np.where(hit, disc, 0))
    # rays clearly inside/outside the silhouette
    clear = np.abs(disc) > 0.05
    assert np.array_equal((fh["tri"] >= 0)[clear], hit[clear])
    sag = r * (1 - math.cos(math.pi / 128))
    m = hit & clear
    cos_inc = np.sqrt(np.maximum(disc[m], 0)) / r
    assert np.all(fh["t"][m] >= t_an[m] - 1e-9)                   # the mesh is inside the sphere
    assert np.all(fh["t"][m] - t_an[m] <= sag / cos_inc + 1e-9)


# ----------------------------------------------------------------------------
# P3: zero return beyond max range (eq.5, Section II-D)
# ----------------------------------------------------------------------------
def _wall(x, rho, sigma=0.0):
    v = [[x, -500, -500], [x, 500, -500], [x, 500, 500], [x, -500, 500]]
    return _scene(v, [[0, 1, 2], [0, 2, 3]], spectra=np.full((1, 61), rho, np.float32), sigma=sigma)


def test_zero_return_beyond_max_range():
    dmax = 50.0
    sensor = S.Sensor(np.array([0.0]), 4, d_max=dmax, az0_deg=-0.0, noise_on=True)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    # wall at d_max + 7 sigma: beyond the largest noise excursion, never seen
    r = O.simulate(_wall(dmax + 7 * 0.02, 0.95, sigma=0.02), sensor, pose, seed=3)
    assert r["valid"][0] == 0 and r["label"][0] == O.MISS_LABEL
    assert r["intensity"][0] == 0 and r["x"][0] == 0 and r["range"][0] == 0
    # wall just beyond d_max with rho > R_L,max: eq.5 alone would pass, the cutoff drops it
    sensor0 = S.Sensor(np.array([0.0]), 4, d_max=dmax, noise_on=False)
    r = O.simulate(_wall(dmax + 1e-3, 0.95), sensor0, pose)
    assert 0.8 / dmax * (dmax + 1e-3) <= 0.95
    assert r["valid"][0] == 0 and r["intensity"][0] == 0 and r["label"][0] == O.MISS_LABEL
    # rho cos = R_L,max: detection up to d_max inclusive (powers of two make
    # R_L(d_max) = R_L,max exact, so this pins the <= comparator and d <= d_max)
    s64 = S.Sensor(np.array([0.0]), 4, d_max=64.0, r_l_max=0.5, noise_on=False)
    r = O.simulate(_wall(64.0, 0.5), s64, pose)
    assert r["t_hit"][0] == 64.0 and r["r_lambda"][0] == 0.5
    assert r["valid"][0] == 1 and r["intensity"][0] == 0.5
    r = O.simulate(_wall(64.0, 0.5 - 2 ** -20), s64, pose)
    assert r["valid"][0] == 0
    r = O.simulate(_wall(dmax * 0.999, 0.8), sensor0, pose)
    assert r["valid"][0] == 1          # R_L(0.999 d_max) = 0.7992 <= 0.8
    r = O.simulate(_wall(dmax * 0.999, 0.79), sensor0, pose)
    assert r["valid"][0] == 0          # 0.7992 > 0.79
    r = O.simulate(_wall(dmax * 0.5, 0.399), sensor0, pose)
    assert r["valid"][0] == 0          # 0.8/50 * 25 = 0.4 > 0.399


def test_noise_added_before_capability_test():
    """Depth noise is added before eq.5 and the cutoff (Section II-D: d includes the noise)."""
    dmax, sig = 50.0, 0.5
    sensor = S.Sensor(np.array([0.0]), 1, d_max=dmax, noise_on=True)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    seen_in, seen_out = 0, 0
    for seed in range(60):
        r = O.simulate(_wall(dmax - 0.3, 0.95, sigma=sig), sensor, pose, seed=seed)
        zd, _ = O.beam_normals(seed, 0, 0, [0])
        dn = (dmax - 0.3) + sig * zd[0]
        assert abs(r["t_hit"][0] - (dmax - 0.3)) < 1e-4
        assert bool(r["valid"][0]) == (dn <= dmax)
        if r["valid"][0]:
            assert abs(r["range"][0] - dn) < 1e-4
            seen_in += 1
        else:
            seen_out += 1
    assert seen_in > 5 and seen_out > 5


def _kat_zero_words():
    """Philox4x32-10 of counter (0, 0, 0, 0) under key (0, 0): the first published known-answer vector."""
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    vec = kat["vectors"][0]
    assert vec["counter"] == ["00000000"] * 4 and vec["key"] == ["00000000"] * 2
    return [int(x, 16) for x in vec["out"]]


def _bm_by_hand(xa, xb):
    """Box-Muller of two 32-bit words written out with math: u1 = (xa + 1) 2^-32, u2 = xb 2^-32."""
    u1 = (xa + 1) / 4294967296.0
    u2 = xb / 4294967296.0
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def _yawed_wall_case(sigma_i, sigma_r=0.02):
    """Beam 0 (elevation 0, azimuth 0) of a sensor yawed by 30 degrees hits the wall x = 10 (rho 0.5)
    at t = 10 / cos 30 with cos(theta) = cos 30; seed 0, scan 0, instance 0 make its Philox block the
    all-zero known-answer vector."""
    sensor = S.Sensor(np.array([0.0]), 4, d_max=50.0, noise_on=True, sigma_intensity=sigma_i)
    q = S.quat_from_ypr(math.radians(30.0))
    pose = S.Pose(np.zeros(3, np.float32), np.asarray(q, np.float32))
    return _wall(10.0, 0.5, sigma=sigma_r), sensor, pose


def test_intensity_noise_uses_words_2_3_and_clamps_at_zero():
    """Intensity noise (a reading: the paper has range noise only): I = max(0, R_lambda + sigma_I z_I)
    with z_I from Philox words 2-3 of counter (beam, scan, instance, 0); range noise from words 0-1."""
    w = _kat_zero_words()
    z_d, z_i = _bm_by_hand(w[0], w[1]), _bm_by_hand(w[2], w[3])
    assert abs(z_d - z_i) > 0.5 and z_i < -0.5          # a swap of the word pairs, or a sign, shows
    for sigma_i in (0.0, 0.05, 0.3):
        scene, sensor, pose = _yawed_wall_case(sigma_i)
        r = O.simulate(scene, sensor, pose, seed=0, scan=0, inst=0, beams=[0])
        # the pose rounds to FP32, so cos(theta) and t are those of the FP32 quaternion's yaw
        d = O.rotation_from_quat(pose.q) @ np.array([1.0, 0.0, 0.0])
        cos_t, t = d[0], 10.0 / d[0]
        assert abs(cos_t - math.cos(math.radians(30.0))) < 1e-7
        r_lam = 0.5 * cos_t
        assert r["valid"][0] == 1
        assert abs(r["r_lambda"][0] - r_lam) < 1e-12
        assert abs(r["range"][0] - (t + 0.02 * z_d)) < 1e-9
        assert abs(r["intensity"][0] - max(0.0, r_lam + float(np.float32(sigma_i)) * z_i)) < 1e-12
    # sigma_I large enough that R_lambda + sigma_I z_I < 0: the clamp gives exactly 0, and the
    # point is still detected (the eq.5 test uses the noise-free R_lambda)
    scene, sensor, pose = _yawed_wall_case(1.0)
    r = O.simulate(scene, sensor, pose, seed=0, scan=0, inst=0, beams=[0])
    assert 0.5 * math.cos(math.radians(30.0)) + 1.0 * z_i < 0.0
    assert r["valid"][0] == 1 and r["intensity"][0] == 0.0 and r["range"][0] > 0.0
    # no noise at all: the intensity is R_lambda whatever sigma_I says
    sensor.noise_on = False
    r = O.simulate(scene, sensor, pose, seed=0, scan=0, inst=0, beams=[0])
    assert abs(r["intensity"][0] - 0.5 * math.cos(math.radians(30.0))) < 1e-7


def test_echo_intensity_noise_uses_words_2_3_and_clamps_at_zero():
    """The multi-echo path draws echo e's noise from counter (beam, scan, instance, e): with one
    sub-ray and no divergence, echo 0 of beam 0 at seed 0 uses the all-zero known-answer block."""
    w = _kat_zero_words()
    z_d, z_i = _bm_by_hand(w[0], w[1]), _bm_by_hand(w[2], w[3])
    for sigma_i in (0.05, 1.0):
        scene, sensor, pose = _yawed_wall_case(sigma_i)
        e = O.simulate_echoes(scene, sensor, pose, n_sub=1, max_echoes=1, divergence_rad=0.0, echo_sep_m=0.5,
                              seed=0, scan=0, beams=[0])
        d = O.rotation_from_quat(pose.q) @ np.array([1.0, 0.0, 0.0])
        r_lam = 0.5 * d[0]
        assert e["valid"][0, 0] == 1
        assert abs(e["range"][0, 0] - (10.0 / d[0] + 0.02 * z_d)) < 1e-9
        assert abs(e["intensity"][0, 0] - max(0.0, r_lam + float(np.float32(sigma_i)) * z_i)) < 1e-12
    assert e["intensity"][0, 0] == 0.0


# ----------------------------------------------------------------------------
# P4: invariance under a rigid transform of scene + sensor
# ----------------------------------------------------------------------------
def test_rigid_transform_invariance():
    scene, sensor, pose = S.small_16ch()
    rng = np.random.default_rng(11)
    beams = rng.choice(sensor.n_beams, 1500, replace=False)
    r0 = O.simulate(scene, sensor, pose, seed=9, beams=beams)
    axis = np.array([0.3, -0.5, 0.8])
    axis /= np.linalg.norm(axis)
    Q = O.so3_exp(0.7 * axis)
    tr = np.array([10.0, -20.0, 5.0])
    v2 = (scene.vertices.astype(np.float64) @ Q.T + tr)
    scene2 = S.Scene(v2.astype(np.float32), scene.indices, scene.material, scene.label,
                     scene.spectra, scene.sigma_range, scene.angle_exp)
    # float32 re-rounding of the moved vertices perturbs geometry by ~1e-6 m; compare
    # away from edges (the FP64 comparison uses the exact transform of the pose)
    R2 = Q @ O.rotation_from_quat(pose.q)
    p2 = Q @ pose.p.astype(np.float64) + tr
    r1 = O.simulate(scene2, sensor, pose, seed=9, beams=beams, R=R2, p=p2)
    ok = ~(r0["ambiguous"] | r1["ambiguous"])
    assert ok.sum() > 1400
    assert np.array_equal(r0["tri"][ok], r1["tri"][ok])
    assert np.array_equal(r0["label"][ok], r1["label"][ok])
    h = ok & r0["hit"]
    assert np.allclose(r0["t_hit"][h], r1["t_hit"][h], rtol=1e-6)
    assert np.allclose(r0["cos_theta"][h], r1["cos_theta"][h], atol=1e-6)
    assert np.allclose(r0["r_lambda"][h], r1["r_lambda"][h], atol=1e-6)
    # exact transform in FP64 (no re-rounding): rotate the pose only, scene fixed,
    # and rotate the beams back -> identical rays, identical results
    r2 = O.simulate(scene, sensor, pose, seed=9, beams=beams,
                    R=O.rotation_from_quat(pose.q), p=pose.p.astype(np.float64))
    assert np.array_equal(r0["tri"], r2["tri"]) and np.array_equal(r0["valid"], r2["valid"])


# ----------------------------------------------------------------------------
# P7: brute force on tiny inputs against an independent algorithm
# ----------------------------------------------------------------------------
def _independent_first_hit(o, d, V, tmin, tmax):
    """Plane intersection + same-side edge tests (not Moller-Trumbore), pure Python."""
    best = (math.inf, -1)
    for k, (a, b, c) in enumerate(V):
        n = np.cross(b - a, c - a)
        den = np.dot(n, d)
        if den == 0:
            continue
        t = np.dot(n, a - o) / den
        if not (tmin < t <= tmax):
            continue
        P = o + t * d
        s1 = np.dot(np.cross(b - a, P - a), n)
        s2 = np.dot(np.cross(c - b, P - b), n)
        s3 = np.dot(np.cross(a - c, P - c), n)
        if s1 >= 0 and s2 >= 0 and s3 >= 0 and (t, k) < best:
            best = (t, k)
    return best


def test_brute_force_matches_independent_algorithm():
    rng = np.random.default_rng(3)
    V = rng.uniform(-5, 5, size=(40, 3, 3))
    scene = _scene(V.reshape(-1, 3), np.arange(120).reshape(40, 3))
    Vf = scene.vertices.astype(np.float64).reshape(40, 3, 3)
    o = np.array([0.1, -0.2, 0.3])
    dirs = rng.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    fh = O.first_hit(scene, o[None], dirs, 0.01, 100.0)
    n_hit = 0
    for r in range(len(dirs)):
        t, k = _independent_first_hit(o, dirs[r], Vf, 0.01, 100.0)
        if fh["edge_in"][r] < 1e-9 or fh["t_second"][r] - fh["t"][r] < 1e-9:
            continue
        assert fh["tri"][r] == k
        if k >= 0:
            n_hit += 1
            assert abs(fh["t"][r] - t) < 1e-9 * max(1, t)
    assert n_hit > 100


def test_tie_break_smaller_index_and_t_min():
    # the same triangle twice (indices 1 and 2) in front of another (index 0) farther away
    v = [[5, -1, -1], [5, 1, -1], [5, 0, 1], [2, -1, -1], [2, 1, -1], [2, 0, 1]]
    scene = _scene(v, [[0, 1, 2], [3, 4, 5], [5, 3, 4]])
    fh = O.first_hit(scene, np.zeros((1, 3)), np.array([[1.0, 0, 0]]), 0.01, 100)
    assert fh["tri"][0] == 1 and fh["t"][0] == 2.0 and fh["t_second"][0] == 2.0
    # t_min excludes surfaces closer than it; t_max excludes farther ones (inclusive)
    fh = O.first_hit(scene, np.zeros((1, 3)), np.array([[1.0, 0, 0]]), 2.0, 100)
    assert fh["tri"][0] == 0
    fh = O.first_hit(scene, np.zeros((1, 3)), np.array([[1.0, 0, 0]]), 0.01, 1.999)
    assert fh["tri"][0] == -1
    fh = O.first_hit(scene, np.zeros((1, 3)), np.array([[1.0, 0, 0]]), 2.0, 5.0)
    assert fh["tri"][0] == 0
    # two-sided: reversed ray from the far side hits too
    fh = O.first_hit(scene, np.array([[10.0, 0, 0]]), np.array([[-1.0, 0, 0]]), 0.01, 100)
    assert fh["tri"][0] == 0 and abs(fh["t"][0] - 5.0) < 1e-12


def test_ambiguity_flags():
    # two triangles sharing the edge x = 0 of a square at z = 0
    v = [[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]]
    scene = _scene(v, [[0, 1, 2], [0, 2, 3]])
    o = np.array([[0.3, 0.3, 5.0], [0.5, -0.2, 5.0], [1.0 + 5e-7, 0.2, 5.0], [1.1, 0.2, 5.0]])
    d = np.array([[0, 0, -1.0]] * 4)
    fh = O.first_hit(scene, o, d, 0.01, 100)
    # on the diagonal: both triangles hit at the same t, edge distance 0
    assert fh["tri"][0] == 0 and fh["t_second"][0] == 5.0 and fh["edge_in"][0] < 1e-12
    # well inside triangle 0 (x > y): clean
    assert fh["tri"][1] == 0 and np.isinf(fh["t_second"][1]) and fh["edge_in"][1] > 0.1
    # just outside the square's edge x = 1: near miss, no hit
    assert fh["tri"][2] == -1 and np.isfinite(fh["near_t"][2])
    # clearly outside: nothing
    assert fh["tri"][3] == -1 and np.isinf(fh["near_t"][3])


# ----------------------------------------------------------------------------
# spectral look-up at the sensor wavelength (Section II-C)
# ----------------------------------------------------------------------------
def test_spectral_interpolation_and_clamp():
    T = np.arange(61, dtype=np.float64)[None, :] * np.array([[1.0], [2.0]])
    r, c = O.reflectance_at_wavelength(T, 850.0)
    assert np.allclose(r, [45, 90]) and not c
    r, c = O.reflectance_at_wavelength(T, 905.0)
    assert np.allclose(r, [50.5, 101]) and not c
    r, c = O.reflectance_at_wavelength(T, 1550.0)
    assert np.allclose(r, [60, 120]) and c
    r, c = O.reflectance_at_wavelength(T, 300.0)
    assert np.allclose(r, [0, 0]) and c
    r, c = O.reflectance_at_wavelength(T, 1000.0)
    assert np.allclose(r, [60, 120]) and not c


def test_label_and_material_of_hit_object():
    scene, sensor, pose = S.small_16ch()
    r = O.simulate(scene, sensor, pose, seed=1)
    h = r["hit"]
    assert np.array_equal(r["label"][r["valid"] == 1], scene.label[r["tri"][r["valid"] == 1]])
    assert np.array_equal(r["material"][h], scene.material[r["tri"][h]])
    assert np.all(r["label"][r["valid"] == 0] == O.MISS_LABEL)
    # every point lies on the ray at its range, sensor frame
    xyz = np.stack([r["x"], r["y"], r["z"]], -1)
    assert np.allclose(np.linalg.norm(xyz, axis=1), r["range"], rtol=1e-12)


# ----------------------------------------------------------------------------
# P8: adjoint of the calibration loss (hit triangles fixed)
# ----------------------------------------------------------------------------
def _calib_problem(n_beams=3000, seed=0):
    cal = S.calibration_20mat()
    scene, sensor = cal["scene"], cal["sensor"]
    rng = np.random.default_rng(seed)
    beams = np.sort(rng.choice(sensor.n_beams, n_beams, replace=False))
    fwd = O.simulate(scene, sensor, cal["pose_true"], beams=beams, rho=cal["rho_true"], angle_exp=cal["k_true"])
    keep = (fwd["valid"] == 1) & ~fwd["ambiguous"] & ~fwd["grazing"]
    return cal, beams[keep], fwd["tri"][keep], fwd["intensity"][keep], fwd["range"][keep]


def test_adjoint_matches_central_differences():
    cal, beams, tri, I_t, t_t = _calib_problem()
    scene, sensor, pose = cal["scene"], cal["sensor"], cal["pose_true"]
    rho = cal["rho0"].astype(np.float64) + 0.05 * np.arange(20) / 20
    kexp = cal["k0"].astype(np.float64) + 0.3 * np.sin(np.arange(20))
    dp = np.array(cal["dp0"]) * 0.05
    dw = np.array(cal["dw0"]) * 0.05
    args = (scene, sensor, pose, tri, beams)
    g_rho, g_k, g_pose = O.calib_grad(*args, rho, kexp, dp, dw, I_t, t_t)
    g = np.concatenate([g_rho, g_k, g_pose])
    h = 1e-6
    fd = np.zeros(46)
    for i in range(46):
        x = np.concatenate([rho, kexp, dp, dw])
        x[i] += h
        lp = O.calib_loss(*args, x[:20], x[20:40], x[40:43], x[43:46], I_t, t_t)
        x[i] -= 2 * h
        lm = O.calib_loss(*args, x[:20], x[20:40], x[40:43], x[43:46], I_t, t_t)
        fd[i] = (lp - lm) / (2 * h)
    for sl in (slice(0, 20), slice(20, 40), slice(40, 43), slice(43, 46)):
        err = np.linalg.norm(g[sl] - fd[sl]) / np.linalg.norm(fd[sl])
        assert err < 1e-4, (sl, err)


def test_calibration_forward_is_the_scan_with_the_triangle_fixed():
    """With the hit triangles held fixed, the calibration forward at the hidden parameters reproduces
    the scan the targets came from: I = the scan's R_lambda (cos^k with k != 1), t = its hit
    distance, at a rotated and displaced pose; so the loss there is 0."""
    cal, beams, tri, I_t, t_t = _calib_problem(n_beams=2000, seed=3)
    scene, sensor, pose = cal["scene"], cal["sensor"], cal["pose_true"]
    rho, kexp = cal["rho_true"].astype(np.float64), cal["k_true"].astype(np.float64)
    assert np.all(np.abs(kexp - 1.0) > 1e-3)           # exponents away from the Lambertian value
    fwd = O.simulate(scene, sensor, pose, beams=beams, rho=rho, angle_exp=kexp)
    s = O.beam_directions(sensor).reshape(-1, 3)[beams]
    I, t, n, d, c, m, live = O._fixed_triangle_forward(scene, s, tri, O.rotation_from_quat(pose.q),
                                                       np.asarray(pose.p, np.float64), rho, kexp)
    assert np.all(live) and np.all(fwd["tri"] == tri)
    assert np.all(np.abs(np.abs(c) - 1.0) > 1e-3)      # oblique incidence, where the exponent matters
    assert np.allclose(I, fwd["r_lambda"], rtol=1e-12, atol=0)
    assert np.allclose(t, fwd["t_hit"], rtol=1e-12, atol=0)
    zero = np.zeros(3)
    assert O.calib_loss(scene, sensor, pose, tri, beams, rho, kexp, zero, zero, I_t, t_t) < 1e-20
    # and not 0 one step away from it, in every group
    for bump in ((0.01, 0, 0, 0), (0, 0.01, 0, 0), (0, 0, 0.01, 0), (0, 0, 0, 0.001)):
        L = O.calib_loss(scene, sensor, pose, tri, beams, rho + bump[0], kexp + bump[1], zero + bump[2],
                         zero + bump[3], I_t, t_t)
        assert L > 1e-9, bump


def test_adjoint_with_intensity_noise_clamp_matches_central_differences():
    """I = max(0, R_lambda + sigma_I z_I): where the clamp holds, I does not move with rho, k or the
    pose.  The analytic gradient (g_I zeroed there) against central differences of the clamped loss,
    with a sigma_I that clamps a good share of the beams."""
    cal, beams, tri, I_t, t_t = _calib_problem(n_beams=1500, seed=4)
    scene, sensor, pose = cal["scene"], cal["sensor"], cal["pose_true"]
    _, z_i = O.beam_normals(77, 0, 0, beams)
    sig_i = 0.25
    rho = cal["rho0"].astype(np.float64) + 0.05 * np.arange(20) / 20
    kexp = cal["k0"].astype(np.float64) + 0.3 * np.sin(np.arange(20))
    dp, dw = np.array(cal["dp0"]) * 0.05, np.array(cal["dw0"]) * 0.05
    s = O.beam_directions(sensor).reshape(-1, 3)[beams]
    R = O.so3_exp(dw) @ O.rotation_from_quat(pose.q)
    I, *_, live = O._fixed_triangle_forward(scene, s, tri, R, np.asarray(pose.p, np.float64) + dp, rho, kexp,
                                            sig_i, z_i)
    assert 0.1 < np.mean(~live) < 0.9 and np.all(I[~live] == 0.0)
    args = (scene, sensor, pose, tri, beams)
    g = np.concatenate(O.calib_grad(*args, rho, kexp, dp, dw, I_t, t_t, sig_i=sig_i, z_i=z_i))
    g_free = np.concatenate(O.calib_grad(*args, rho, kexp, dp, dw, I_t, t_t))
    h = 1e-6
    fd = np.zeros(46)
    for i in range(46):
        x = np.concatenate([rho, kexp, dp, dw])
        x[i] += h
        lp = O.calib_loss(*args, x[:20], x[20:40], x[40:43], x[43:46], I_t, t_t, sig_i=sig_i, z_i=z_i)
        x[i] -= 2 * h
        lm = O.calib_loss(*args, x[:20], x[20:40], x[40:43], x[43:46], I_t, t_t, sig_i=sig_i, z_i=z_i)
        fd[i] = (lp - lm) / (2 * h)
    for sl in (slice(0, 20), slice(20, 40), slice(40, 43), slice(43, 46)):
        err = np.linalg.norm(g[sl] - fd[sl]) / np.linalg.norm(fd[sl])
        assert err < 1e-4, (sl, err)
        # ignoring the clamp is wrong by far more than the tolerance (the translation has no
        # intensity term)
        assert np.linalg.norm(g_free[sl] - fd[sl]) / np.linalg.norm(fd[sl]) > 1e-3 or sl == slice(40, 43), sl


def test_adjoint_special_cases():
    # beam straight down onto the ground plane from 10 m: c = -1
    scene = _ground(spectra=np.full((1, 61), 0.4, np.float32))
    sensor = S.Sensor(np.array([-90.0]), 1, noise_on=False)
    pose = S.Pose(np.array([0, 0, 10.0], np.float32), np.array([1, 0, 0, 0], np.float32))
    beams = np.array([0])
    tri = np.array([0])
    zero = np.zeros(3)
    # L = (I - I*)^2 with I* = I - 1 -> g_I = 2: dL/drho = 2 cos^k = 2, dL/dk = 0 (ln 1 = 0)
    rho, k = np.array([0.4]), np.array([1.7])
    g_rho, g_k, g_pose = O.calib_grad(scene, sensor, pose, tri, beams, rho, k, zero, zero,
                                      np.array([0.4 - 1.0]), np.array([10.0]), lam_d=0.0)
    assert abs(g_rho[0] - 2.0) < 1e-12 and abs(g_k[0]) < 1e-12
    # depth only, t* = t - 1 -> g_t = 2; dt/dp = -n/c = +z here (moving up lengthens the ray)
    g_rho, g_k, g_pose = O.calib_grad(scene, sensor, pose, tri, beams, rho, k, zero, zero,
                                      np.array([0.4]), np.array([9.0]), lam_d=1.0)
    assert np.allclose(g_pose[:3], [0, 0, 2.0], atol=1e-9)
    assert np.allclose(g_pose[3:], 0, atol=1e-9)


def test_spectral_adjoint_matches_central_differences_on_the_table():
    """dL/dT[m, b] through the interpolation at the sensor wavelength, against
    central differences of the loss with R_lambda(0) re-read from the perturbed
    table: on a bin centre, between bins, and clamped below and above the table."""
    import dataclasses
    cal, beams, tri, I_t, t_t = _calib_problem(n_beams=1500, seed=1)
    scene, pose = cal["scene"], cal["pose_true"]
    T = scene.spectra.astype(np.float64)
    kexp = cal["k0"].astype(np.float64) + 0.2
    dp, dw = np.array(cal["dp0"]) * 0.05, np.array(cal["dw0"]) * 0.05
    for lam, hot in ((900.0, (50,)), (905.0, (50, 51)), (931.0, (53, 54)), (380.0, (0,)), (1550.0, (60,))):
        sensor = dataclasses.replace(cal["sensor"], wavelength_nm=lam)
        args = (scene, sensor, pose, tri, beams)
        g_T, g_k, g_pose = O.calib_grad_spectral(*args, T, kexp, dp, dw, I_t, t_t)
        rho_of = lambda TT: O.reflectance_at_wavelength(TT, lam)[0]   # noqa: E731
        g_rho, g_k2, g_pose2 = O.calib_grad(*args, rho_of(T), kexp, dp, dw, I_t, t_t)
        assert np.array_equal(g_k, g_k2) and np.array_equal(g_pose, g_pose2)
        cold = [b for b in (0, 10, 25, 49, 52, 55, 59, 60) if b not in hot]
        h = 1e-6
        for m in (0, 3, 11):
            for b in list(hot) + cold[:3]:
                Tp, Tm = T.copy(), T.copy()
                Tp[m, b] += h
                Tm[m, b] -= h
                lp = O.calib_loss(*args, rho_of(Tp), kexp, dp, dw, I_t, t_t)
                lm = O.calib_loss(*args, rho_of(Tm), kexp, dp, dw, I_t, t_t)
                fd = (lp - lm) / (2 * h)
                assert abs(g_T[m, b] - fd) <= 1e-6 * max(1.0, abs(fd)), (lam, m, b, g_T[m, b], fd)
        assert np.count_nonzero(g_T.sum(axis=0)) == len(hot)
        assert np.all(g_T[:, [b for b in range(61) if b not in hot]] == 0)
