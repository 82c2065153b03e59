"""Pins of the oracle's partial-sweep (per-tick, rolling-shutter) path against
closed forms and brute force, independent of the oracle's own formulas.

Section II-A: at every engine tick only the part of FOV_h swept by the spinning
head since the previous tick is simulated (from the spin rate and the tick
length).  Each fired column takes the pose of its firing time.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S


def _sensor(n_az, fov=360.0, az0=0.0, elev=(-10.0, 0.0, 10.0), **kw):
    return S.Sensor(np.array(elev), n_az, az0_deg=az0, fov_h_deg=fov, **kw)


def _fired(runs):
    return [(s, i) for s, lo, hi in runs for i in range(lo, hi)]


def test_ticks_partition_revolutions_exactly_once():
    """60 Hz ticks of a 10 Hz head (341.33 columns each) fire every column of
    three revolutions exactly once, in firing order."""
    sensor = _sensor(2048)
    seq = []
    for k in range(18):
        a, b = O.sweep_window(k * 60.0, 10.0, 1.0 / 60.0)
        seq += _fired(O.sweep_columns(sensor, a, b))
    assert seq == [(g // 2048, g % 2048) for g in range(3 * 2048)]


def test_sweep_columns_match_brute_force_in_rational_arithmetic():
    """Random windows (away from exact column angles) against the definition
    a <= 360 s + az0 + i FOV_h / N_az < b evaluated exactly with fractions."""
    rng = np.random.default_rng(11)
    for n_az, fov, az0 in ((7, 200.0, 10.0), (16, 360.0, 0.0), (5, 90.0, -30.0), (1, 360.0, 45.0)):
        sensor = _sensor(n_az, fov, az0)
        for _ in range(200):
            a = float(rng.uniform(-400.0, 1500.0))
            b = a + float(rng.uniform(0.0, 360.0))
            runs = O.sweep_columns(sensor, a, b)
            want = []
            for s in range(0, 8):
                for i in range(n_az):
                    A = 360 * s + Fraction(az0) + i * Fraction(fov) / n_az
                    if Fraction(a) <= A < Fraction(b):
                        want.append((s, i))
            assert _fired(runs) == want, (n_az, fov, az0, a, b)


def test_sweep_columns_at_exact_column_angles():
    """Window ends on exactly representable column angles: the start column is
    fired, the end column is not."""
    sensor = _sensor(8)                      # columns every 45 degrees
    assert _fired(O.sweep_columns(sensor, 45.0, 135.0)) == [(0, 1), (0, 2)]
    assert _fired(O.sweep_columns(sensor, 315.0, 405.0)) == [(0, 7), (1, 0)]
    assert O.sweep_columns(sensor, 100.0, 100.0) == []
    assert _fired(O.sweep_columns(sensor, 0.0, 360.0)) == [(0, i) for i in range(8)]
    with pytest.raises(ValueError):
        O.sweep_columns(sensor, 0.0, 361.0)


def _quat_axis_angle(axis, ang):
    axis = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    return np.r_[math.cos(ang / 2.0), math.sin(ang / 2.0) * axis]


def test_slerp_is_constant_speed_rotation_about_the_common_axis():
    """Rotations about one axis by angles a and b: slerp at tau is the rotation
    about that axis by a + tau (b - a), whichever sign the quaternions carry."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        axis = rng.normal(size=3)
        a, b = rng.uniform(-1.5, 1.5, size=2)
        qa, qb = _quat_axis_angle(axis, a), _quat_axis_angle(axis, b)
        if rng.uniform() < 0.5:
            qb = -qb                          # same rotation, other hemisphere
        for tau in (0.0, 0.25, 0.5, 0.9, 1.0):
            got = O.rotation_from_quat(O.slerp(qa, qb, tau))
            want = O.so3_exp(np.asarray(axis) / np.linalg.norm(axis) * (a + tau * (b - a)))
            np.testing.assert_allclose(got, want, atol=1e-13)


def test_slerp_of_equal_ends_is_exactly_that_quaternion():
    q = np.array([0.9, 0.1, -0.3, 0.2])
    for tau in (0.0, 0.3, 1.0):
        assert np.array_equal(O.slerp(q, q, tau), q)
        assert np.array_equal(O.slerp(q, -q, tau), q)      # same rotation, other sign


def _wall_scene(x_wall):
    v = np.array([[x_wall, -500, -500], [x_wall, 500, -500], [x_wall, 0, 500]], np.float32)
    return S.Scene(v, np.array([[0, 1, 2]], np.uint32), np.array([0], np.uint16), np.array([7], np.uint32),
                   np.full((1, 61), 0.9, np.float32), np.array([0.0], np.float32), np.array([1.0], np.float32))


def test_rolling_shutter_translation_closed_form():
    """Sensor moving along +x at v towards the wall x = X: the horizontal beam at
    azimuth theta (|theta| < 60 deg) fires at t = (theta - a) / (360 omega) after the
    tick start and measures (X - v t) / cos(theta)."""
    X, v, spin, dt = 40.0, 12.0, 10.0, 1.0 / 30.0      # a third of a revolution per tick
    sensor = _sensor(720, elev=(0.0,), d_max=200.0, noise_on=False)
    a0 = -60.0 + 360.0                                   # tick over [300, 420) degrees of revolution 0/1
    pa = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    pb = S.Pose(np.array([v * dt, 0, 0], np.float32), np.array([1, 0, 0, 0], np.float32))
    o = O.simulate_sweep(_wall_scene(X), sensor, pa, pb, a0, spin, dt)
    assert [r[0] for r in o["runs"]] == [0, 1]
    col = o["beams"] % sensor.n_az
    theta = np.where(o["scan"] == 0, col * 0.5 + 0.0, col * 0.5 + 360.0)   # unwrapped head angle
    t_fire = (theta - a0) / (360.0 * spin)
    want = (X - float(np.float32(v * dt)) / dt * t_fire) / np.cos(np.deg2rad(theta))
    assert np.all(o["valid"] == 1)
    np.testing.assert_allclose(o["range"], want, rtol=1e-12)
    np.testing.assert_allclose(o["tau"], t_fire / dt, rtol=0, atol=1e-12)


def test_rolling_shutter_rotation_closed_form():
    """Sensor yawing at a constant rate during the tick: the world direction of
    the beam (phi, theta) fired at tau is the sensor direction turned by
    yaw_a + tau (yaw_b - yaw_a) about z."""
    sensor = _sensor(64, elev=(-20.0, 5.0, 30.0), noise_on=False)
    ya, yb = 0.3, 0.3 + math.radians(20.0)
    pa = S.Pose(np.zeros(3, np.float32), S.quat_from_ypr(ya))
    pb = S.Pose(np.zeros(3, np.float32), S.quat_from_ypr(yb))
    o = O.simulate_sweep(_wall_scene(30.0), sensor, pa, pb, 100.0, 5.0, 0.1)   # 180 degrees
    qa = np.asarray(pa.q, np.float64)
    qb = np.asarray(pb.q, np.float64)
    # the float32 quaternions are rotations about z by 2 atan2(qz, qw)
    ya32, yb32 = 2 * math.atan2(qa[3], qa[0]), 2 * math.atan2(qb[3], qb[0])
    j, i = o["beams"] // sensor.n_az, o["beams"] % sensor.n_az
    phi = np.deg2rad(sensor.elev_deg[j])
    yaw = ya32 + o["tau"] * (yb32 - ya32)
    th = np.deg2rad(i * (360.0 / 64)) + yaw
    want = np.stack([np.cos(phi) * np.cos(th), np.cos(phi) * np.sin(th), np.sin(phi)], axis=1)
    np.testing.assert_allclose(o["dir_world"], want, atol=1e-12)
    assert np.all(np.diff(o["tau"][j == 0]) > 0) and o["tau"].min() >= 0 and o["tau"].max() < 1


def test_constant_pose_ticks_reproduce_the_full_scan():
    """Ticks with one pose covering revolution 2 give exactly the outputs of
    the full scan with scan counter 2 (same rays, same Philox counters)."""
    scene, sensor, pose = S.small_16ch()
    pose = S.Pose(pose.p, S.quat_from_ypr(0.7, 0.05, -0.03))
    full = O.simulate(scene, sensor, pose, seed=77, scan=2)
    got = {k: np.zeros_like(full[k]) for k in ("valid", "range", "label", "tri", "intensity", "x", "y", "z")}
    n = 0
    for k in range(7):                                  # 7 ticks of 360/7 degrees
        o = O.simulate_sweep(scene, sensor, pose, pose, 720.0 + k * (360.0 / 7), 10.0, 1.0 / 70.0, seed=77)
        n += len(o["beams"])
        assert np.all(o["scan"] == 2)
        for key in got:
            got[key][o["beams"]] = o[key]
    assert n == sensor.n_beams
    for key in got:
        assert np.array_equal(got[key], full[key]), key
