"""GPU parity of divergent beams with multi-echo returns (the paper's named
future work; model as read in the oracle) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import compare_echoes, to_np

pytestmark = pytest.mark.gpu

SEED = 0xEC40


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


def _ctx(L, scene, sensor, pose):
    c = L.Context(0)
    c.load(scene)
    c.set_sensor(sensor)
    c.set_pose(pose.p, pose.q)
    return c


def _np(out):
    return {k: (v.cpu().numpy().view(np.uint32) if k in ("tri", "label") else
                v.cpu().numpy().view(np.uint16) if k == "material" else v.cpu().numpy()) for k, v in out.items()}


def test_one_subray_is_the_single_return_bit_for_bit(L):
    scene, sensor, pose = S.urban_64ch()
    c = _ctx(L, scene, sensor, pose)
    single = to_np(c.simulate(SEED, 3, debug=True))
    e = _np(c.simulate_echoes(SEED, 3, 1, 2, 0.0, 0.5, debug=True))
    for k in ("valid", "label", "x", "y", "z", "intensity", "range", "tri", "t_hit", "material", "r_lambda"):
        assert np.array_equal(e[k][0], single[k]), k
    assert not e["valid"][1].any() and np.all(e["tri"][1] == 0xFFFFFFFF)


def test_echoes_match_oracle_full_16ch(L):
    scene, sensor, pose = S.small_16ch()
    pose = S.Pose(pose.p, S.quat_from_ypr(0.3, 0.01, 0.0))
    c = _ctx(L, scene, sensor, pose)
    g = _np(c.simulate_echoes(SEED, 1, 16, 4, 0.01, 0.3, debug=True))
    c.sync_check()
    o = O.simulate_echoes(scene, sensor, pose, 16, 4, float(np.float32(0.01)), float(np.float32(0.3)),
                          seed=SEED, scan=1)
    rep = compare_echoes(g, o)
    print(f"[parity] echoes 16ch K=16: {rep}", flush=True)
    assert rep["detected"][0] > 3000 and rep["echoes_formed"][1] > 100


def test_echoes_match_oracle_sampled_64ch(L):
    scene, sensor, pose = S.urban_64ch()
    c = _ctx(L, scene, sensor, pose)
    g = _np(c.simulate_echoes(SEED, 0, 7, 3, 0.003, 0.5, debug=True))
    rng = np.random.default_rng(4)
    multi = np.flatnonzero(g["tri"][1] != 0xFFFFFFFF)
    beams = np.unique(np.r_[rng.choice(sensor.n_beams, 2000, replace=False),
                            rng.choice(multi, min(1000, len(multi)), replace=False)])
    o = O.simulate_echoes(scene, sensor, pose, 7, 3, float(np.float32(0.003)), 0.5, seed=SEED, scan=0, beams=beams)
    rep = compare_echoes({k: v[:, beams] for k, v in g.items()}, o)
    print(f"[parity] echoes 64ch K=7 sampled: {rep}", flush=True)
    assert rep["detected"][1] > 10


def test_echo_launch_shapes_agree(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    ref = None
    for tile, lanes in ((16, 4), (1, 2), (64, 1), (4, 4)):
        c.set_tile_shape(tile)
        c.set_lanes_per_ray(lanes)
        g = _np(c.simulate_echoes(SEED, 2, 9, 3, 0.02, 0.25, debug=True))
        if ref is None:
            ref = g
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (tile, lanes, k)


def test_echoes_with_actors_match_oracle(L):
    cfg = S.dynamic_actors()
    c = _ctx(L, cfg["scene"], cfg["sensor"], cfg["pose"])
    for m in cfg["meshes"]:
        c.load_mesh(m)
    acts = cfg["actors_at"](0.5)
    c.set_actors(acts)
    g = _np(c.simulate_echoes(SEED, 0, 7, 2, 0.003, 0.5, debug=True))
    on_actor = np.flatnonzero(g["label"][0] >= 100000)
    rng = np.random.default_rng(6)
    beams = np.unique(np.r_[rng.choice(cfg["sensor"].n_beams, 800, replace=False),
                            rng.choice(on_actor, min(700, len(on_actor)), replace=False)])
    soup, _ = O.scene_with_actors(cfg["scene"], cfg["meshes"], acts)
    o = O.simulate_echoes(soup, cfg["sensor"], cfg["pose"], 7, 2, float(np.float32(0.003)), 0.5, seed=SEED,
                          beams=beams)
    rep = compare_echoes({k: v[:, beams] for k, v in g.items()}, o)
    print(f"[parity] echoes with actors: {rep}", flush=True)


def test_echo_argument_errors(L):
    from paper_2208_10295_amd import _abi as A
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    for bad in ((0, 1, 0.0, 0.5), (17, 1, 0.0, 0.5), (4, 5, 0.0, 0.5), (4, 2, -1.0, 0.5), (4, 2, 0.01, 0.0)):
        with pytest.raises(L.LidarError):
            c.simulate_echoes(0, 0, *bad)
    d = A.EchoDesc(4, 2, 0.01, 0.5)
    out = c.simulate_echoes(0, 0, 4, 2, 0.01, 0.5)
    small = torch.empty(1024, dtype=torch.uint8, device=c.device)
    o = L.lidar.outputs_struct({k: v.reshape(-1) for k, v in out.items()})
    assert A.lib.lidar_simulate_echoes(c.h, 0, 0, d, small.data_ptr(), 1024, o, None) == A.ERR_WORKSPACE_TOO_SMALL
    n = c.simulate_echoes(0, 0, 4, 2, 0.01, 0.5, debug=True)
    assert "normal" not in n
