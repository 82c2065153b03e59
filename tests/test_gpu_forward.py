"""GPU parity of the forward path (trace + return model) against the FP64 oracle.

All calls go through the C ABI (liblidar.so) via the thin Python binding.
"""
import math

import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu

SEED = 0x1234_5678_9ABC


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


def _ctx(L, scene, sensor, pose, leaf_width=4):
    c = L.Context(0)
    c.load(scene, leaf_width)
    c.set_sensor(sensor)
    c.set_pose(pose.p, pose.q)
    return c


def _report(name, rep):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v}" for k, v in rep.items()), flush=True)


def test_16ch_full_scan_matches_oracle(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    g = to_np(c.simulate(SEED, scan=3, debug=True))
    c.sync_check()
    o = O.simulate(scene, sensor, pose, seed=SEED, scan=3)
    rep = compare(g, o)
    _report("small_16ch full", rep)
    assert rep["valid"] > 3000 and rep["ambiguous"] < 0.01 * rep["n"]


def test_16ch_bvh_equals_bruteforce_and_is_deterministic(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    a = to_np(c.simulate(SEED, 1, debug=True))
    b = to_np(c.simulate(SEED, 1, debug=True, bruteforce=True))
    a2 = to_np(c.simulate(SEED, 1, debug=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], a2[k]), k


def test_launch_shapes_do_not_change_results(L):
    """Leaf width, tile shape, lanes per ray and the XCD remap change speed only."""
    scene, sensor, pose = S.small_16ch()
    ref = None
    for W in (1, 2, 3, 4, 8):
        c = _ctx(L, scene, sensor, pose, leaf_width=W)
        shapes = ([(t, l, x) for t in (1, 8, 64) for l in (1, 2, 4) for x in (0, 1)] if W == 4
                  else [(8, 4, 1), (8, 1, 0), (4, 2, 1)])
        for tile, lanes, xcd in shapes:
            c.set_tile_shape(tile)
            c.set_lanes_per_ray(lanes)
            c.set_xcd_remap(xcd)
            g = to_np(c.simulate(SEED, 0, debug=True))
            if ref is None:
                ref = g
            for k in ref:
                assert np.array_equal(ref[k], g[k]), (W, tile, lanes, xcd, k)


def test_64ch_full_scan_matches_oracle_every_beam(L):
    """The 64 x 2048 scan of the 522,272-triangle scene, every one of its 131,072 beams against the FP64
    brute-force oracle (6.85e10 ray-triangle tests, about 13 s on 16 host threads)."""
    scene, sensor, pose = S.urban_64ch()
    c = _ctx(L, scene, sensor, pose)
    st = c.stats()
    print("[bvh] urban_64ch", st, flush=True)
    out = c.simulate(SEED, scan=0, debug=True)
    c.sync_check()
    o = O.simulate(scene, sensor, pose, seed=SEED, scan=0)
    rep = compare(to_np(out), o)
    _report("urban_64ch every beam", rep)
    assert rep["n"] == 131072 and rep["tri_mismatch"] == 0 and rep["valid_mismatch"] == 0
    assert rep["valid"] > 50000 and rep["ambiguous"] < 0.01 * rep["n"]


def test_64ch_bvh_equals_bruteforce_full(L):
    """Both tree builders, both collapses, trees built for rays near the horizontal (horizontal faces weighted
    0.5 and 0.15 in the area metric) and every traversal shape reproduce the brute-force scan bit for bit."""
    scene, sensor, pose = S.urban_64ch()
    c = _ctx(L, scene, sensor, pose)
    b = to_np(c.simulate(SEED, 0, debug=True, bruteforce=True))
    for builder, collapse, upw in (("ploc", "sah", 1.0), ("lbvh", "sah", 1.0), ("ploc", "greedy", 1.0),
                                   ("lbvh", "greedy", 1.0), ("ploc", "sah", 0.5), ("ploc", "sah", 0.15)):
        st = c.load(scene, builder=builder, collapse=collapse, up_weight=upw)
        print(f"[bvh] urban_64ch {builder} {collapse} up {upw}: nodes {st['n_nodes']} leaves {st['n_leaves']} "
              f"depth {st['depth']} build {st['build_ms']:.2f} ms", flush=True)
        for lanes in (1, 2, 4):
            c.set_lanes_per_ray(lanes)
            a = to_np(c.simulate(SEED, 0, debug=True))
            for k in a:
                assert np.array_equal(a[k], b[k]), (builder, collapse, upw, lanes, k)


@pytest.mark.parametrize("builder,collapse,leaf_width,leaf_cost,up_weight", [
    ("ploc", "sah", 4, 0.0, 1.0), ("lbvh", "sah", 4, 0.0, 1.0), ("ploc", "greedy", 4, 0.0, 1.0),
    ("lbvh", "greedy", 4, 0.0, 1.0), ("ploc", "sah", 1, 0.0, 1.0), ("ploc", "sah", 8, 0.0, 1.0),
    ("lbvh", "sah", 2, 0.0, 1.0), ("ploc", "sah", 4, 0.25, 1.0), ("ploc", "sah", 4, 8.0, 1.0),
    ("ploc", "sah", 4, 0.0, 0.25), ("lbvh", "sah", 2, 0.0, 1.0 / 128)])
def test_bvh_structure_invariants(L, builder, collapse, leaf_width, leaf_cost, up_weight):
    """Every triangle lies in exactly one leaf of at most leaf_width triangles, and every child box contains
    its triangles, for each builder and collapse (a very cheap and a very dear leaf step, and area metrics
    that weight the horizontal faces down to 1/128, included)."""
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    c.load(scene, leaf_width, builder=builder, collapse=collapse, leaf_cost=leaf_cost, up_weight=up_weight)
    st = c.stats()
    assert st["leaf_width"] == leaf_width
    nodes_b, tris_b = c.debug_bvh()
    nodes = nodes_b.view(np.float32).reshape(-1, 4, 8)
    refs = nodes_b.view(np.uint32).reshape(-1, 4, 8)[:, :, 3]
    recs = tris_b.view(np.float32).reshape(-1, 12)
    orig = tris_b.view(np.uint32).reshape(-1, 12)[:, 3]
    assert sorted(orig.tolist()) == list(range(scene.n_tri))
    seen = np.zeros(scene.n_tri, np.int64)
    reached = np.zeros(st["n_nodes"], np.int64)
    stack = [0]
    reached[0] = 1
    while stack:
        nd = stack.pop()
        for k in range(4):
            ref = int(refs[nd, k])
            if ref == 0xFFFFFFFF:
                continue
            lo, hi = nodes[nd, k, 0:3], nodes[nd, k, 4:7]
            if ref & 0x80000000:
                first, cnt = (ref >> 3) & 0x0FFFFFFF, (ref & 7) + 1
                assert cnt <= st["leaf_width"]
                seen[first:first + cnt] += 1
                v = recs[first:first + cnt][:, [0, 1, 2, 4, 5, 6, 8, 9, 10]].reshape(-1, 3)
                assert np.all(v >= lo) and np.all(v <= hi)
            else:
                assert 0 < ref < st["n_nodes"] and reached[ref] == 0
                reached[ref] = 1
                stack.append(ref)
    assert np.all(seen == 1) and np.all(reached == 1)



def _collapse_cost(nodes_b, pad, leaf_cost):
    """Surface-area cost of a 4-wide tree with the collapse's weights: 1 x area per node below the root,
    leaf_cost x area x ceil(count / 4) per leaf, in FP64 on the stored child boxes with their pad removed."""
    f = nodes_b.view(np.float32).reshape(-1, 4, 8).astype(np.float64)
    refs = nodes_b.view(np.uint32).reshape(-1, 4, 8)[:, :, 3]
    e = np.maximum((f[:, :, 4:7] - pad) - (f[:, :, 0:3] + pad), 0.0)
    area = e[..., 0] * e[..., 1] + e[..., 1] * e[..., 2] + e[..., 2] * e[..., 0]
    used = refs != 0xFFFFFFFF
    leaf = used & ((refs & 0x80000000) != 0)
    inner = used & ~leaf
    steps = ((refs & 7) + 1 + 3) // 4
    return float((area * inner).sum() + leaf_cost * (area * steps * leaf).sum())


@pytest.mark.parametrize("builder,leaf_width", [("ploc", 4), ("lbvh", 4), ("ploc", 8), ("lbvh", 1)])
def test_cost_shaped_collapse_is_no_worse_than_greedy(L, builder, leaf_width):
    """The bottom-up programme minimises the surface-area cost over every 4-wide collapse of the binary
    tree, and the greedy collapse is one of them: the cost of the default tree cannot exceed the greedy
    tree's (same builder, same binary tree; the two share only the binary tree)."""
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    cost = {}
    for collapse in ("sah", "greedy"):
        st = c.load(scene, leaf_width, builder=builder, collapse=collapse)
        cost[collapse] = _collapse_cost(c.debug_bvh()[0], float(st["box_pad"]), 1.5)
    print(f"[collapse] {builder} W={leaf_width}: cost sah {cost['sah']:.6g} greedy {cost['greedy']:.6g}", flush=True)
    # the programme sums in FP32 and the unpadded boxes are rounded: a relative 1e-4 covers both
    assert cost["sah"] <= cost["greedy"] * (1 + 1e-4)

def test_ragged_sensor_and_offsets(L):
    """Odd channel/azimuth counts, a partial FOV and a scene far from the origin."""
    scene, _, _ = S.small_16ch()
    off = np.array([3000.0, -1500.0, 40.0])
    sc2 = S.Scene((scene.vertices.astype(np.float64) + off).astype(np.float32), scene.indices, scene.material,
                  scene.label, scene.spectra, scene.sigma_range, scene.angle_exp)
    sensor = S.Sensor(np.array([-14.0, -9.5, -3.0, 0.5, 7.0]), 37, az0_deg=10.0, fov_h_deg=200.0, d_max=80.0)
    pose = S.Pose((np.array([0.0, 0.0, 1.5]) + off).astype(np.float32), S.quat_from_ypr(0.3, 0.02, -0.01))
    c = _ctx(L, sc2, sensor, pose)
    o = O.simulate(sc2, sensor, pose, seed=99, scan=5)
    for tile in (1, 4, 64):
        for lanes in (1, 2, 4):
            c.set_tile_shape(tile)
            c.set_lanes_per_ray(lanes)
            g = to_np(c.simulate(99, 5, debug=True))
            _report(f"ragged tile {tile} lanes {lanes}", compare(g, o))


def test_single_triangle_scene(L):
    v = np.array([[10, -5, -5], [10, 5, -5], [10, 0, 5]], np.float32)
    scene = S.Scene(v, np.array([[0, 1, 2]], np.uint32), np.array([0], np.uint16), np.array([42], np.uint32),
                    np.full((1, 61), 0.6, np.float32), np.array([0.0], np.float32), np.array([1.0], np.float32))
    sensor = S.Sensor(np.array([-10.0, 0.0, 10.0]), 16, d_max=50.0, noise_on=False)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    c = _ctx(L, scene, sensor, pose)
    assert c.stats()["n_nodes"] == 1
    g = to_np(c.simulate(0, 0, debug=True))
    o = O.simulate(scene, sensor, pose)
    compare(g, o)
    assert g["valid"][16 * 1 + 0] == 1 and g["label"][16] == 42
    assert abs(g["range"][16] - 10.0) < 1e-5 and abs(g["intensity"][16] - 0.6) < 1e-6


def test_128ch_5m_sequence_256_beams_of_every_scan(L):
    """The 100-scan trajectory in the 5,224,200-triangle scene: 256 seeded beams of each of the 100 scans
    (25,600 beams, 1.3e11 ray-triangle tests) against the oracle, each scan with its own pose and Philox
    scan counter."""
    scene, sensor, poses = S.urban_sequence_128ch()
    c = L.Context(0)
    st = c.load(scene)
    print("[bvh] urban_sequence_128ch", st, flush=True)
    c.set_sensor(sensor)
    rng = np.random.default_rng(3)
    tot = {}
    for scan, pose in enumerate(poses):
        c.set_pose(pose.p, pose.q)
        out = c.simulate(SEED, scan, debug=True)
        beams = np.sort(rng.choice(sensor.n_beams, 256, replace=False))
        o = O.simulate(scene, sensor, pose, seed=SEED, scan=scan, beams=beams)
        rep = compare(to_np(out, beams), o)
        for k, v in rep.items():
            tot[k] = max(tot.get(k, 0), v) if k.endswith("_max_rel") else tot.get(k, 0) + v
    c.sync_check()
    _report("urban_sequence_128ch, 256 beams x 100 scans", tot)
    assert tot["n"] == 25600 and tot["tri_mismatch"] == 0 and tot["valid_mismatch"] == 0 and tot["valid"] > 5000


def test_wavelength_clamp_warning_and_values(L):
    scene, sensor, pose = S.small_16ch()
    s2 = S.Sensor(sensor.elev_deg, 64, wavelength_nm=1550.0, d_max=100.0)
    c = L.Context(0)
    c.load(scene)
    with pytest.warns(RuntimeWarning):
        c.set_sensor(s2)
    c.set_pose(pose.p, pose.q)
    g = to_np(c.simulate(5, 0, debug=True))
    o = O.simulate(scene, s2, pose, seed=5)
    assert o["wavelength_clamped"]
    compare(g, o)


def test_degenerate_triangles_and_axis_aligned_beams(L):
    """Zero-area triangles (a repeated vertex, collinear vertices, all three equal) are never hit and do not
    change any other beam; beams exactly along the axes (elevation 0, azimuths 0/90/180/270 deg: two zero
    direction components) hit axis-aligned walls, including a wall edge, as the oracle and the brute force
    say."""
    def box(x0, y0, z0, x1, y1, z1):
        v = [[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0], [x0, y0, z1], [x1, y0, z1], [x1, y1, z1],
             [x0, y1, z1]]
        t = [[0, 1, 2], [0, 2, 3], [4, 6, 5], [4, 7, 6], [0, 4, 5], [0, 5, 1], [1, 5, 6], [1, 6, 2], [2, 6, 7],
             [2, 7, 3], [3, 7, 4], [3, 4, 0]]
        return np.array(v, np.float64), np.array(t)
    parts = [box(-60, -60, -3, 60, 60, -2), box(8, -2, -1, 9, 2, 1), box(-2, 12, -1, 2, 13, 1),
             box(-15, 0, -1, -14, 2, 1), box(-1, -21, -1, 1, -20, 1)]   # the -x wall's edge is at y = 0
    good_v, good_t, nv = [], [], 0
    for v, t in parts:
        good_v.append(v)
        good_t.append(t + nv)
        nv += len(v)
    gv = np.concatenate(good_v)
    gt = np.concatenate(good_t)
    # degenerate triangles, placed where the axis beams pass
    dv = np.array([[5, -1, 0], [5, 1, 0], [5, 1, 0],            # repeated vertex
                   [0, 6, -1], [0, 6, 0], [0, 6, 1],            # collinear along z, on the +y beam
                   [-7, 0, 0], [-7, 0, 0], [-7, 0, 0]], np.float64)   # a point on the -x beam
    dt = np.arange(9).reshape(3, 3) + len(gv)
    def scene_of(v, t):
        nt = len(t)
        return S.Scene(v.astype(np.float32), t.astype(np.uint32), np.zeros(nt, np.uint16),
                       np.arange(1, nt + 1, dtype=np.uint32), np.full((1, 61), 0.7, np.float32),
                       np.array([0.0], np.float32), np.array([1.0], np.float32))
    with_deg = scene_of(np.concatenate([gv, dv]), np.concatenate([gt, dt]))
    without = scene_of(gv, gt)
    sensor = S.Sensor(np.array([-30.0, -5.0, 0.0, 5.0]), 8, d_max=50.0, noise_on=False)
    pose = S.Pose(np.zeros(3, np.float32), np.array([1, 0, 0, 0], np.float32))
    ca = _ctx(L, with_deg, sensor, pose)
    a = to_np(ca.simulate(0, 0, debug=True))
    b = to_np(ca.simulate(0, 0, debug=True, bruteforce=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    cw = _ctx(L, without, sensor, pose)
    w = to_np(cw.simulate(0, 0, debug=True))
    for k in a:
        assert np.array_equal(a[k], w[k]), k            # the degenerate triangles change nothing
    assert not np.isin(a["tri"], np.arange(len(gt), len(gt) + 3)).any()     # no degenerate triangle is hit
    o = O.simulate(with_deg, sensor, pose)
    _report("degenerate + axis beams", compare(a, o))
    # elevation-0 beams at azimuths 0, 90, 180, 270 deg (every second of 8 steps): walls at x = 8 (through
    # the diagonal shared by the face's two triangles: a tie, the smaller index wins), y = 12, x = -14 (on
    # the wall's lower edge, y = 0) and y = -20
    j0 = 2 * 8
    for i, t in ((0, 8.0), (2, 12.0), (4, 14.0), (6, 20.0)):
        assert a["valid"][j0 + i] == 1 and abs(a["range"][j0 + i] - t) < 1e-5 * t, (i, a["range"][j0 + i])


def test_stack_overflow_is_reported_and_recovered(L):
    """The overflow path, forced from the host: with the stack capped at one entry every walk that needs a
    second one loses children, stays within its stack memory and ends; sync_check reports the overflow,
    and with the cap lifted the same scan is bit-identical to the uncapped one."""
    from paper_2208_10295_amd import _abi as A
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    ref = to_np(c.simulate(SEED, 0, debug=True))
    c.sync_check()
    for lanes in (1, 2, 4):
        c.set_lanes_per_ray(lanes)
        c.set_stack_cap(1)
        print(f"[overflow] lanes={lanes} cap=1", flush=True)
        c.simulate(SEED, 0, debug=True)
        with pytest.raises(L.LidarError) as e:
            c.sync_check()
        assert e.value.status == A.ERR_STACK_OVERFLOW
        c.set_stack_cap(0)
        g = to_np(c.simulate(SEED, 0, debug=True))
        c.sync_check()
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (lanes, k)
    # a cap the walks never reach changes nothing
    c.set_stack_cap(30)
    g = to_np(c.simulate(SEED, 0, debug=True))
    c.sync_check()
    for k in ref:
        assert np.array_equal(ref[k], g[k]), k
    with pytest.raises(L.LidarError):
        c.set_stack_cap(-1)


def test_range_and_intensity_noise_are_independent_standard_normals(L):
    """The noise the kernel adds (Philox4x32-10 words through Box-Muller, Section II-A range noise and the
    intensity noise) is standard normal and independent between range and intensity: z_d = (d - t) / sigma_m
    and z_I = (I - R_lambda) / sigma_I over the beams whose detection and clamp the noise cannot change."""
    import dataclasses
    from scipy import stats
    scene, sensor, pose = S.urban_64ch()
    sensor = dataclasses.replace(sensor, sigma_intensity=0.01)
    c = _ctx(L, scene, sensor, pose)
    g = to_np(c.simulate(SEED, 3, debug=True))
    mat = g["material"].astype(np.int64)
    sig = np.asarray(scene.sigma_range, np.float64)[np.minimum(mat, len(scene.sigma_range) - 1)]
    t, d, rl, inten = (g[k].astype(np.float64) for k in ("t_hit", "range", "r_lambda", "intensity"))
    # far from the eq.5 limit, the range cutoff and the intensity clamp at 0 (more than 8 sigma)
    safe = ((g["valid"] == 1) & (sig > 0) & (t < 0.8 * sensor.d_max) &
            (rl > (sensor.r_l_max / sensor.d_max) * (t + 8 * sig) * 1.01) & (rl > 8 * sensor.sigma_intensity))
    assert safe.sum() > 20000
    zd = (d[safe] - t[safe]) / sig[safe]
    zi = (inten[safe] - rl[safe]) / sensor.sigma_intensity
    print(f"[noise] n={safe.sum()} z_d mean {zd.mean():.4f} std {zd.std():.4f}; "
          f"z_I mean {zi.mean():.4f} std {zi.std():.4f}; corr {np.corrcoef(zd, zi)[0, 1]:.4f}", flush=True)
    for z in (zd, zi):
        assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03
        assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(zd, zi)[0, 1]) < 0.03


def test_trajectory_launcher_equals_pose_then_simulate(L):
    """The per-tick trajectory launcher (pose k, then scan k, argument structs built once) gives the same
    outputs bit for bit as setting each pose and simulating scan k."""
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    poses = [S.Pose((np.asarray(pose.p, np.float64) + [0.7 * k, -0.3 * k, 0.0]).astype(np.float32),
                    S.quat_from_ypr(0.2 * k, 0.01 * k, 0.0)) for k in range(3)]
    from paper_2208_10295_amd.lidar import alloc_outputs, POINT_OUTPUTS
    out = alloc_outputs(sensor.n_beams, POINT_OUTPUTS, c.device)
    run = c.trajectory_launcher(SEED, out, poses)
    for k in (2, 0, 1):
        run(k)
        got = to_np({key: v.clone() for key, v in out.items()})
        c.set_pose(poses[k].p, poses[k].q)
        ref = to_np(c.simulate(SEED, k))
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (k, key)


def test_origin_outside_the_padded_cube_warns(L):
    """The box padding covers FP32 rounding for origins inside the cube |x|,|y|,|z| <= M (M the largest
    |vertex coordinate|): a pose, a sweep end, a batch instance or a scene loaded under a pose outside
    it gives the warning, and the call still does its work."""
    from paper_2208_10295_amd import _abi as A
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    M = float(c.stats()["max_abs_coord"])
    assert M == float(np.max(np.abs(scene.vertices[scene.indices.astype(np.int64)])))
    assert c.set_pose(pose.p, pose.q) == A.OK
    far = np.array([1.2 * M, 0.0, 1.5], np.float32)      # 20 % beyond the ground's edge, 1.5 m up
    with pytest.warns(RuntimeWarning, match="outside the cube"):
        st = c.set_pose(far, pose.q)
    assert st & A.WARN_ORIGIN_OUTSIDE_SCENE
    g = to_np(c.simulate(0, 0, debug=True))  # still simulated: the beams towards the scene hit it
    assert (g["tri"] != 0xFFFFFFFF).sum() > 100
    with pytest.warns(RuntimeWarning, match="outside the cube"):
        c.load(scene)
    with pytest.warns(RuntimeWarning, match="outside the cube"):
        c.simulate_sweep(1, 0.0, 10.0, 1 / 60, (pose.p, pose.q), (far, pose.q))
    b = c.batch([S.Instance(sensor, pose), S.Instance(sensor, S.Pose(far, pose.q))], 64)
    assert b.origin_outside and not c.batch([S.Instance(sensor, pose)], 64).origin_outside
