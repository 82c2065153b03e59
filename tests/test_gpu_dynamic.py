"""GPU parity of dynamic scenes (meshes placed by moving actors, one labelled
instance each, Section II-B) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu

SEED = 0xD1_7A


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


@pytest.fixture(scope="module")
def dyn(L):
    cfg = S.dynamic_actors()
    ctx = L.Context(0)
    ctx.load(cfg["scene"])
    ctx.set_sensor(cfg["sensor"])
    ctx.set_pose(cfg["pose"].p, cfg["pose"].q)
    ids = [ctx.load_mesh(m) for m in cfg["meshes"]]
    assert ids == list(range(len(cfg["meshes"])))
    return ctx, cfg


def _sample(g, sensor, rng, n=2500):
    """Random beams plus beams whose GPU hit is an actor (so actor hits are always covered)."""
    on_actor = np.flatnonzero(g["label"] >= 100000)
    pick = rng.choice(on_actor, min(len(on_actor), 1500), replace=False) if len(on_actor) else []
    return np.unique(np.r_[rng.choice(sensor.n_beams, n, replace=False), pick]).astype(np.int64)


def test_dynamic_scene_matches_oracle(L, dyn):
    ctx, cfg = dyn
    sensor = cfg["sensor"]
    actors = cfg["actors_at"](0.0)
    ctx.set_actors(actors)
    g = to_np(ctx.simulate(SEED, 0, debug=True))
    ctx.sync_check()
    n_actor_hits = int((g["label"] >= 100000).sum())
    assert n_actor_hits > 500
    beams = _sample(g, sensor, np.random.default_rng(1))
    o = O.simulate_actors(cfg["scene"], cfg["meshes"], actors, sensor, cfg["pose"], seed=SEED, scan=0, beams=beams)
    rep = compare({k: v[..., beams] for k, v in g.items()}, o)
    print(f"[parity] dynamic t=0: {rep}, actor hits in the scan {n_actor_hits}", flush=True)
    assert rep["valid"] > 1000


def test_update_refit_equals_rebuild_and_oracle(L, dyn):
    """With the builder's top-level tree, moving the actors by lidar_actors_update
    (refit) gives the outputs of a rebuild with lidar_actors_set, bit for bit, and
    matches the oracle."""
    ctx, cfg = dyn
    sensor = cfg["sensor"]
    ctx.set_actor_tree(1)
    try:
        ctx.set_actors(cfg["actors_at"](0.0))
        for t in (0.4, 1.3):
            acts = cfg["actors_at"](t)
            ctx.update_actors(acts)
            a = to_np(ctx.simulate(SEED, 1, debug=True))
            ctx.set_actors(acts)
            b = to_np(ctx.simulate(SEED, 1, debug=True))
            for k in a:
                assert np.array_equal(a[k], b[k]), (t, k)
    finally:
        ctx.set_actor_tree(0)
    beams = _sample(a, sensor, np.random.default_rng(2), n=1500)
    o = O.simulate_actors(cfg["scene"], cfg["meshes"], acts, sensor, cfg["pose"], seed=SEED, scan=1, beams=beams)
    rep = compare({k: v[..., beams] for k, v in a.items()}, o)
    print(f"[parity] dynamic t=1.3 (refit): {rep}", flush=True)


def _scan_with_tree(ctx, mode, acts, scan=3):
    ctx.set_actor_tree(mode)
    try:
        ctx.set_actors(acts)
        return to_np(ctx.simulate(SEED, scan, debug=True))
    finally:
        ctx.set_actor_tree(0)


def test_packed_tree_equals_builder_tree(L, dyn):
    """The top-level tree rebuilt by every update (Morton-packed, one workgroup)
    and the builder's tree give the same outputs bit for bit: on frames reached by
    updates far from the first frame's positions, and for actor sets of 1 to 17
    actors (trees of one and two levels, partly empty nodes)."""
    ctx, cfg = dyn
    ctx.set_actor_tree(0)
    ctx.set_actors(cfg["actors_at"](0.0))
    t = 0.0
    for t_next in (0.9, 2.5):
        while t < t_next - 1e-9:
            t = round(t + 0.1, 6)
            ctx.update_actors(cfg["actors_at"](t))
        a = to_np(ctx.simulate(SEED, 3, debug=True))
        b = _scan_with_tree(ctx, 1, cfg["actors_at"](t))
        ctx.set_actors(cfg["actors_at"](t))        # the packed tree again, for the next updates
        for k in a:
            assert np.array_equal(a[k], b[k]), (t, k)
        assert (a["label"] >= 100000).sum() > 500
    every = cfg["actors_at"](0.3)
    near = np.argsort([float(np.hypot(x.p[0], x.p[1])) for x in every])
    on_actors = 0
    for n in (1, 2, 4, 5, 17):
        acts = [every[k] for k in near[:n]]
        a = _scan_with_tree(ctx, 0, acts)
        b = _scan_with_tree(ctx, 1, acts)
        for k in a:
            assert np.array_equal(a[k], b[k]), (n, k)
        on_actors += int((a["label"] >= 100000).sum())
    assert on_actors > 0


@pytest.mark.parametrize("n_act", [1024, 1025, 4096])
def test_packed_tree_large_sets(L, n_act):
    """The rebuild's two orderings at their limits, against the builder's tree: up to
    1,024 actors (one per thread, each placed by counting smaller keys) and above
    (bitonic sort), up to 4,096 actors, the most one workgroup rebuilds (a 6-level
    tree of 1,365 nodes)."""
    n_peds = n_act // 4
    cfg = S.dynamic_actors(seed=77, n_cars=n_act - n_peds, n_peds=n_peds)
    ctx = L.Context(0)
    ctx.load(cfg["scene"])
    ctx.set_sensor(cfg["sensor"])
    ctx.set_pose(cfg["pose"].p, cfg["pose"].q)
    for m in cfg["meshes"]:
        ctx.load_mesh(m)
    acts = cfg["actors_at"](0.5)
    assert len(acts) == n_act
    ctx.set_actors(cfg["actors_at"](0.0))
    ctx.update_actors(acts)
    a = to_np(ctx.simulate(SEED, 0, debug=True))
    ctx.sync_check()
    b = _scan_with_tree(ctx, 1, acts, scan=0)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert (a["label"] >= 100000).sum() > 1000


def test_updates_on_several_streams(L, dyn):
    """Updates issued on alternating streams (the upload ring wraps) leave the tree a fresh set at the last
    poses gives, bit for bit."""
    ctx, cfg = dyn
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx.set_actors(cfg["actors_at"](0.0))
    for f in range(1, 20):
        ctx.update_actors(cfg["actors_at"](0.1 * f), stream=s1 if f % 3 else s2)
    torch.cuda.synchronize()
    a = to_np(ctx.simulate(SEED, 4, debug=True))
    ctx.set_actors(cfg["actors_at"](1.9))
    b = to_np(ctx.simulate(SEED, 4, debug=True))
    ctx.sync_check()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_mesh_refit_equals_fresh_build(L, dyn):
    """A deformed pedestrian mesh refit in place scans like the deformed mesh built from scratch."""
    ctx, cfg = dyn
    acts = cfg["actors_at"](0.7)
    ped = cfg["meshes"][3]
    sway = S.pedestrian_pose_vertices(ped, 1.1)
    ctx.set_actors(acts)
    ctx.refit_mesh(3, sway)
    with pytest.raises(L.LidarError):
        ctx.simulate(SEED, 0)                      # the actors' boxes are stale until the update
    ctx.update_actors(acts)
    a = to_np(ctx.simulate(SEED, 0, debug=True))
    fresh = L.Context(0)
    fresh.load(cfg["scene"])
    fresh.set_sensor(cfg["sensor"])
    fresh.set_pose(cfg["pose"].p, cfg["pose"].q)
    for m in cfg["meshes"][:3] + [S.Mesh(sway, ped.indices, ped.material)]:
        fresh.load_mesh(m)
    fresh.set_actors(acts)
    b = to_np(fresh.simulate(SEED, 0, debug=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    on_ped = np.flatnonzero((a["label"] >= 100200) & (a["label"] < 100300))
    assert len(on_ped) > 10
    beams = np.unique(np.r_[on_ped[:600], np.random.default_rng(3).choice(cfg["sensor"].n_beams, 500)])
    o = O.simulate_actors(cfg["scene"], cfg["meshes"], acts, cfg["sensor"], cfg["pose"], seed=SEED, beams=beams,
                          mesh_vertices=[None, None, None, sway])
    print("[parity] deformed pedestrians:", compare({k: v[..., beams] for k, v in a.items()}, o), flush=True)
    ctx.refit_mesh(3, ped.vertices)                # back to the rest pose
    ctx.update_actors(acts)


def test_launch_shapes_and_sweep_with_actors(L, dyn):
    ctx, cfg = dyn
    sensor, pose = cfg["sensor"], cfg["pose"]
    ctx.set_actors(cfg["actors_at"](0.2))
    ref = None
    for lanes in (4, 2, 1):
        ctx.set_lanes_per_ray(lanes)
        g = to_np(ctx.simulate(SEED, 2, debug=True))
        if ref is None:
            ref = g
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (lanes, k)
    ctx.set_lanes_per_ray(4)
    out = None
    pq = (pose.p, pose.q)
    head = 2 * 360.0 - 0.05
    for _ in range(6):
        out, _ = ctx.simulate_sweep(SEED, head, 10.0, 1.0 / 60.0, pq, pq, out=out, debug=True)
        head = head + 360.0 * 10.0 * (1.0 / 60.0)
    g = to_np(out)
    for k in ref:
        assert np.array_equal(ref[k], g[k]), ("sweep", k)


def test_static_only_paths_reject_actors_and_clear_restores(L, dyn):
    ctx, cfg = dyn
    ctx.set_actors(cfg["actors_at"](0.0))
    with pytest.raises(L.LidarError):
        ctx.simulate(0, 0, bruteforce=True)
    with pytest.raises(L.LidarError):
        ctx.simulate_counts(0, 0)
    out = ctx.simulate(0, 0, debug=True)
    with pytest.raises(L.LidarError):
        ctx.backward(out["tri"], out["valid"], out["intensity"], out["range"])
    with pytest.raises(L.LidarError):
        ctx.update_actors(cfg["actors_at"](0.1)[:-1])       # the count must not change
    ctx.clear_actors()
    a = to_np(ctx.simulate(SEED, 0, debug=True))
    plain = L.Context(0)
    plain.load(cfg["scene"])
    plain.set_sensor(cfg["sensor"])
    plain.set_pose(cfg["pose"].p, cfg["pose"].q)
    b = to_np(plain.simulate(SEED, 0, debug=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
