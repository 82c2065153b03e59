"""Pins of the oracle's dynamic-scene path (meshes placed by moving actors,
each actor one labelled object instance, Section II-B) against closed forms
and against relations that do not use the oracle's own transform code."""
import math

import numpy as np

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S


def _far_scene(nmat=16):
    """A static scene that no beam of the tests reaches (one small triangle far below)."""
    v = np.array([[0, 0, -900], [1, 0, -900], [0, 1, -900]], np.float32)
    return S.Scene(v, np.array([[0, 1, 2]], np.uint32), np.array([0], np.uint16), np.array([1], np.uint32),
                   np.full((nmat, 61), 0.5, np.float32), np.zeros(nmat, np.float32), np.ones(nmat, np.float32))


def _cube(half=1.0, mat=2):
    v, t = S.box_mesh([-half, -half, -half], [half, half, half])
    return S.Mesh(v.astype(np.float32), t.astype(np.uint32), np.full(len(t), mat, np.uint16))


def test_rotated_cube_closed_form():
    """A 2 m cube yawed by 30 deg, centred 10 m ahead: the horizontal beam at azimuth 0 meets the
    face x' = -1 at t = 10 - 1 / cos 30, incidence cos 30; label = the actor's."""
    scene = _far_scene()
    scene.spectra[2, :] = 0.8
    sensor = S.Sensor(np.array([0.0]), 8, noise_on=False)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    yaw = math.radians(30.0)
    actor = S.Actor(0, 4242, np.array([10.0, 0.0, 0.0], np.float32),
                    np.array([math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)], np.float32))
    o = O.simulate_actors(scene, [_cube()], [actor], sensor, pose)
    # the float32 quaternion is a rotation about z by 2 atan2(qz, qw)
    y32 = 2 * math.atan2(float(actor.q[3]), float(actor.q[0]))
    assert o["valid"][0] == 1 and o["label"][0] == 4242
    assert abs(o["range"][0] - (10.0 - 1.0 / math.cos(y32))) < 1e-12
    assert abs(o["cos_theta"][0] - math.cos(y32)) < 1e-12
    assert abs(o["intensity"][0] - float(np.float32(0.8)) * math.cos(y32)) < 1e-12
    assert o["tri"][0] >= o["tri_base"][0]            # an actor triangle, not the static one
    # the beam at azimuth 180 deg sees nothing
    assert o["valid"][4] == 0


def test_moving_the_actor_equals_moving_the_sensor_inversely():
    """Placing the mesh by (R_a, p_a) and scanning from (R_s, p_s) gives the ranges of the mesh at the
    identity scanned from (R_a^T R_s, R_a^T (p_s - p_a)) (FP64 pose override)."""
    scene = _far_scene()
    mesh = S.car_mesh()
    sensor = S.Sensor(S.elev_table(16), 180, noise_on=False, d_max=60.0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        yaw, pitch, roll = rng.uniform(-math.pi, math.pi), rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2)
        actor = S.Actor(0, 7, rng.uniform(-3, 3, size=3).astype(np.float32), S.quat_from_ypr(yaw, pitch, roll))
        pose = S.Pose(np.array([actor.p[0] + 6.0, actor.p[1] - 2.0, actor.p[2] + 1.0], np.float32),
                      S.quat_from_ypr(rng.uniform(-math.pi, math.pi)))
        o = O.simulate_actors(scene, [mesh], [actor], sensor, pose)
        Ra = O.rotation_from_quat(actor.q)
        Rs = O.rotation_from_quat(pose.q)
        ident = S.Actor(0, 7, np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
        soup, _ = O.scene_with_actors(scene, [mesh], [ident])
        r = O.simulate(soup, sensor, pose, R=Ra.T @ Rs,
                       p=Ra.T @ (np.asarray(pose.p, np.float64) - np.asarray(actor.p, np.float64)))
        ok = ~(o["ambiguous"] | r["ambiguous"])
        assert o["valid"].sum() > 50
        assert np.array_equal(o["tri"][ok], r["tri"][ok]) and np.array_equal(o["valid"][ok], r["valid"][ok])
        np.testing.assert_allclose(o["range"][ok], r["range"][ok], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(o["cos_theta"][ok], r["cos_theta"][ok], rtol=1e-9, atol=1e-9)


def test_ties_go_to_the_static_scene_then_to_the_earlier_actor():
    scene = _far_scene()
    # a static square (2 triangles) exactly where the actors' cube face will be: plane x = 9
    v = np.array([[9, -5, -5], [9, 5, -5], [9, 5, 5], [9, -5, 5]], np.float32)
    st = S.Scene(np.concatenate([scene.vertices, v]), np.array([[0, 1, 2], [3, 4, 5], [3, 5, 6]], np.uint32),
                 np.array([0, 1, 1], np.uint16), np.array([1, 55, 55], np.uint32), scene.spectra, scene.sigma_range,
                 scene.angle_exp)
    sensor = S.Sensor(np.array([0.0]), 8, noise_on=False)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    ident = np.array([1, 0, 0, 0], np.float32)
    a1 = S.Actor(0, 1001, np.array([10.0, 0, 0], np.float32), ident)
    a2 = S.Actor(0, 1002, np.array([10.0, 0, 0], np.float32), ident)
    o = O.simulate_actors(st, [_cube()], [a1, a2], sensor, pose)
    assert o["label"][0] == 55 and o["range"][0] == 9.0
    o = O.simulate_actors(scene, [_cube()], [a1, a2], sensor, pose)
    assert o["label"][0] == 1001 and o["range"][0] == 9.0 and o["amb_tie"][0]


def test_deformed_vertices_are_applied_in_object_space():
    """A mesh whose vertices are shifted by s in object space equals the actor moved by R s."""
    scene = _far_scene()
    mesh = S.pedestrian_mesh()
    sensor = S.Sensor(S.elev_table(16), 360, noise_on=False, d_max=40.0)
    pose = S.Pose(np.array([0, 0, 1.0], np.float32), np.array([1, 0, 0, 0], np.float32))
    q = S.quat_from_ypr(0.9)
    shift = np.array([0.25, -0.5, 0.0])
    a = S.Actor(0, 9, np.array([5.0, 1.0, 0.0], np.float32), q)
    o1 = O.simulate_actors(scene, [mesh], [a], sensor, pose,
                           mesh_vertices=[(mesh.vertices.astype(np.float64) + shift).astype(np.float32)])
    p2 = (np.asarray(a.p, np.float64) + O.rotation_from_quat(q) @ shift).astype(np.float32)
    o2 = O.simulate_actors(scene, [mesh], [S.Actor(0, 9, p2, q)], sensor, pose)
    ok = ~(o1["ambiguous"] | o2["ambiguous"])
    assert o1["valid"].sum() > 20
    assert np.array_equal(o1["tri"][ok], o2["tri"][ok])
    np.testing.assert_allclose(o1["range"][ok], o2["range"][ok], rtol=1e-6)
    # and the sway of the walking pose changes the scan
    sway = O.simulate_actors(scene, [mesh], [a], sensor, pose,
                             mesh_vertices=[S.pedestrian_pose_vertices(mesh, 1.2)])
    assert not np.array_equal(sway["range"], O.simulate_actors(scene, [mesh], [a], sensor, pose)["range"])
