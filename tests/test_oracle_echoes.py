"""Pins of the oracle's divergent-beam, multi-echo path (the paper's conclusion
names beam divergence and multi-echo returns as the next effects to model)
against its single-return special case, closed-form geometry and the Philox
definition."""
import math

import numpy as np

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S


def test_one_subray_without_divergence_is_the_single_return():
    scene, sensor, pose = S.small_16ch()
    pose = S.Pose(pose.p, S.quat_from_ypr(0.4, 0.02, 0.01))
    o = O.simulate(scene, sensor, pose, seed=9, scan=4)
    e = O.simulate_echoes(scene, sensor, pose, 1, 3, 0.0, 0.5, seed=9, scan=4)
    for k in ("valid", "range", "intensity", "label", "x", "y", "z", "tri", "t_hit", "material", "r_lambda"):
        assert np.array_equal(e[k][0], o[k].astype(e[k].dtype)), k
    assert not e["valid"][1:].any() and np.all(e["n_echoes"] <= 1)


def test_subray_pattern_geometry():
    """Sub-ray k leaves the axis by r_k = (delta/2) sqrt(k/(K-1)) in the tangent direction at angle
    b_k = k * golden angle from the azimuth tangent, measured from the computed unit vectors."""
    sensor = S.Sensor(np.array([-20.0, 0.0, 35.0]), 12)
    K, delta = 9, 0.004
    beams = np.arange(sensor.n_beams)
    d = O.subray_directions(sensor, beams, K, delta)
    assert np.allclose(np.linalg.norm(d, axis=-1), 1.0, atol=1e-15)
    th = np.deg2rad(np.arange(12) * 30.0)[beams % 12]
    ph = np.deg2rad(sensor.elev_deg)[beams // 12]
    axis = np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], -1)
    e_th = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], -1)
    e_ph = np.cross(axis, e_th)                 # completes the right-handed frame (axis, e_theta, e_phi)
    assert np.allclose(d[:, 0], axis, atol=1e-15)
    for k in range(1, K):
        ang = np.arccos(np.clip(np.einsum("ij,ij->i", d[:, k], axis), -1, 1))
        assert np.allclose(ang, 0.5 * delta * math.sqrt(k / (K - 1)), atol=1e-9)
        b = np.arctan2(np.einsum("ij,ij->i", d[:, k], e_ph), np.einsum("ij,ij->i", d[:, k], e_th))
        want = math.remainder(k * math.pi * (3 - math.sqrt(5)), 2 * math.pi)
        assert np.allclose(np.remainder(b - want + math.pi, 2 * math.pi) - math.pi, 0, atol=1e-9)


def _plate_and_wall(x_plate, x_wall, rho_plate, rho_wall):
    """A plate at x = x_plate over y >= 0 and a wall at x = x_wall, both facing the sensor."""
    v = np.array([[x_plate, 0, -50], [x_plate, 50, -50], [x_plate, 50, 50], [x_plate, 0, 50],
                  [x_wall, -50, -50], [x_wall, 50, -50], [x_wall, 50, 50], [x_wall, -50, 50]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7]], np.uint32)
    spectra = np.zeros((2, 61), np.float32)
    spectra[0], spectra[1] = rho_plate, rho_wall
    return S.Scene(v, idx, np.array([0, 0, 1, 1], np.uint16), np.array([5, 5, 6, 6], np.uint32), spectra,
                   np.zeros(2, np.float32), np.ones(2, np.float32))


def test_beam_split_by_an_edge_gives_two_echoes_in_closed_form():
    """The horizontal beam at azimuth 0 straddles the plate's edge y = 0: sub-rays with d_y > 0
    meet the plate at t = 10 / d_x (incidence cos = d_x), the others the wall at 20 / d_x."""
    scene = _plate_and_wall(10.0, 20.0, 0.9, 0.7)
    sensor = S.Sensor(np.array([0.0]), 4, noise_on=False, d_max=100.0)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    K, delta = 7, 0.01
    e = O.simulate_echoes(scene, sensor, pose, K, 3, delta, 0.5, beams=[0])
    rho_p, rho_w = float(np.float32(0.9)), float(np.float32(0.7))
    # sub-ray 0 (the axis, d_y = 0) runs along the plate's edge: the beam is flagged ambiguous; move the
    # sensor 1 mm off the edge plane for the closed form
    assert e["ambiguous"][0]
    e = O.simulate_echoes(scene, sensor, S.Pose(np.array([0, -1e-3, 0], np.float32), pose.q), K, 3, delta, 0.5,
                          beams=[0])
    d = O.subray_directions(sensor, [0], K, delta)[0]
    plate = -1e-3 + 10.0 * d[:, 1] / d[:, 0] > 0         # where the sub-ray crosses x = 10
    assert 0 < plate.sum() < K
    for echo, sel, x, rho, lab in ((0, plate, 10.0, rho_p, 5), (1, ~plate, 20.0, rho_w, 6)):
        t = x / d[sel, 0]
        R = rho * d[sel, 0]
        P = R.sum() / K
        te = t[np.argmin(t)] + np.sum(R * (t - t[np.argmin(t)])) / R.sum()
        assert e["valid"][echo, 0] == 1 and e["label"][echo, 0] == lab
        assert abs(e["range"][echo, 0] - te) < 1e-9 and abs(e["intensity"][echo, 0] - P) < 1e-12
    assert e["n_echoes"][0] == 2 and e["valid"][2, 0] == 0


def test_surfaces_closer_than_the_separation_form_one_echo():
    scene = _plate_and_wall(10.0, 10.3, 0.9, 0.7)
    sensor = S.Sensor(np.array([0.0]), 4, noise_on=False)
    pose = S.Pose(np.array([0, -1e-3, 0], np.float32), np.array([1, 0, 0, 0], np.float32))
    e = O.simulate_echoes(scene, sensor, pose, 7, 3, 0.01, 0.5, beams=[0])
    assert e["n_echoes"][0] == 1 and 10.0 < e["range"][0, 0] < 10.3
    e2 = O.simulate_echoes(scene, sensor, pose, 7, 3, 0.01, 0.2, beams=[0])
    assert e2["n_echoes"][0] == 2


def test_echo_noise_uses_the_echo_index_as_the_fourth_counter_word():
    scene = _plate_and_wall(10.0, 20.0, 0.9, 0.9)
    scene.sigma_range[:] = 0.05
    sensor = S.Sensor(np.array([0.0]), 4, noise_on=True, sigma_intensity=0.0)
    pose = S.Pose(np.array([0, -1e-3, 0], np.float32), np.array([1, 0, 0, 0], np.float32))
    seed, scan = 0xABCDEF0123, 7
    noisy = O.simulate_echoes(scene, sensor, pose, 7, 2, 0.01, 0.5, seed=seed, scan=scan, beams=[0])
    quiet = O.simulate_echoes(scene, S.Sensor(np.array([0.0]), 4, noise_on=False), pose, 7, 2, 0.01, 0.5,
                              beams=[0])
    for e in (0, 1):
        x = O.philox4x32_10(np.array([[0, scan, 0, e]], np.uint64), (seed & 0xFFFFFFFF, seed >> 32))[0]
        u1 = (float(x[0]) + 1.0) * 2.0 ** -32
        z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * float(x[1]) * 2.0 ** -32)
        assert abs(noisy["range"][e, 0] - (quiet["range"][e, 0] + float(np.float32(0.05)) * z)) < 1e-12
