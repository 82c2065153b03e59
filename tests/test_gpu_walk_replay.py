"""The CPU walk replay (measure/walk_replay.c) against the GPU on the GPU-built trees.

Per beam, the replay's node fetches and triangle-record tests must equal the GPU counting kernel's
(lidar_simulate_counts, the walk the roofline's algorithmic bytes describe) exactly, and its best hit must
be the GPU's bit for bit: the same original triangle index and the same FP32 distance.  Run on every beam
of the 64 x 2048 scan of the 522k-triangle scene (two and four lanes per beam, whose walks visit the same
nodes in the same order) and on two poses of the 128 x 1024 trajectory in the 5.2M-triangle scene.
"""
import numpy as np
import pytest
import torch

from lidar_inputs import scenes as S
from measure import walk_replay as W
from tests.parity import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


def _check(L, ctx, scene, sensor, pose, seed, scan, tag):
    ctx.set_pose(pose.p, pose.q)
    _, nn, nt = ctx.simulate_counts(seed, scan)
    g = to_np(ctx.simulate(seed, scan, debug=True))
    ctx.sync_check()
    nodes, recs = ctx.debug_bvh()
    st = ctx.stats()
    r = W.replay(nodes, recs, st["root"], sensor, pose.p, pose.q, sensor.t_min,
                 W.trace_limit(sensor, scene.sigma_range), touched=True)
    assert r["not_replayed"] == 0
    gn = nn.cpu().numpy().view(np.uint32)
    gt = nt.cpu().numpy().view(np.uint32)
    bad_n = np.flatnonzero(gn != r["node_visits"])
    bad_t = np.flatnonzero(gt != r["tri_tests"])
    hit = g["tri"] != 0xFFFFFFFF
    assert np.array_equal(hit, r["orig"] != 0xFFFFFFFF), tag
    bad_o = np.flatnonzero(g["tri"] != r["orig"])
    bad_d = np.flatnonzero(hit & (g["t_hit"].view(np.uint32) != r["t"].view(np.uint32)))
    print(f"[replay] {tag}: {sensor.n_beams} beams, nodes/beam {gn.mean():.3f}, records/beam {gt.mean():.3f}, "
          f"distinct nodes {r['nodes_touched']} of {st['n_nodes']}, records {r['records_touched']} of "
          f"{st['n_triangles']}; mismatches: nodes {len(bad_n)}, records {len(bad_t)}, hit {len(bad_o)}, "
          f"t {len(bad_d)}", flush=True)
    assert len(bad_n) == 0 and len(bad_t) == 0 and len(bad_o) == 0 and len(bad_d) == 0, tag
    return r


@pytest.mark.parametrize("lanes", [4, 2])
def test_replay_equals_gpu_counts_on_the_full_64ch_scan(L, lanes):
    scene, sensor, pose = S.urban_64ch()
    ctx = L.Context(0)
    ctx.load(scene)
    ctx.set_sensor(sensor)
    ctx.set_lanes_per_ray(lanes)
    _check(L, ctx, scene, sensor, pose, 2022, 0, f"64x2048, lanes {lanes}")


def test_replay_equals_gpu_counts_on_the_5m_trajectory(L):
    scene, sensor, poses = S.urban_sequence_128ch()
    ctx = L.Context(0)
    ctx.load(scene)
    ctx.set_sensor(sensor)
    for k in (0, 61):
        _check(L, ctx, scene, sensor, poses[k], 7, k, f"128x1024 pose {k}, 5.2M triangles")
