"""GPU parity of the per-tick partial sweep with rolling-shutter poses
(Section II-A: only the part of FOV_h swept since the previous tick is
simulated) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED_0F_71C


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


def _ctx(L, scene, sensor):
    c = L.Context(0)
    c.load(scene)
    c.set_sensor(sensor)
    return c


def _sentinel_outputs(L, n, device="cuda"):
    out = L.alloc_outputs(n, ("x", "y", "z", "intensity", "label", "valid", "range", "tri", "t_hit", "material",
                              "normal", "r_lambda"), device)
    for k, t in out.items():
        if t.dtype == torch.uint8:
            t.fill_(0xA5)
        elif t.dtype in (torch.int32, torch.int16):
            t.fill_(-2)
        else:
            t.fill_(float("nan"))
    return out


def _written(g, sensor):
    """Columns whose every beam was written (valid is 0 or 1, never the fill value)."""
    v = g["valid"].reshape(sensor.n_ch, sensor.n_az)
    w = v != 0xA5
    assert np.all(w.all(axis=0) | (~w).all(axis=0)), "a column was written partly"
    return w.all(axis=0)


def _run_ticks(c, L, sensor, pose, head0, spin, dt, n_ticks, seed):
    out = _sentinel_outputs(L, sensor.n_beams)
    pq = (pose.p, pose.q)
    fired = []
    a = head0
    for _ in range(n_ticks):
        out, runs = c.simulate_sweep(seed, a, spin, dt, pq, pq, out=out)
        fired += [(s, i) for s, f, n in runs for i in range(f, f + n)]
        a = a + 360.0 * spin * dt                   # next tick starts where this one ended
    torch.cuda.synchronize()
    return to_np(out), fired


@pytest.mark.parametrize("cfg", ["small_16ch", "urban_64ch"])
def test_fixed_pose_ticks_equal_the_full_scan_bit_for_bit(L, cfg):
    """Ticks of one revolution at a fixed pose reproduce lidar_simulate(scan)
    exactly (all outputs), and fire every column once."""
    scene, sensor, pose = getattr(S, cfg)()
    pose = S.Pose(pose.p, S.quat_from_ypr(0.7, 0.05, -0.03))
    c = _ctx(L, scene, sensor)
    c.set_pose(pose.p, pose.q)
    full = to_np(c.simulate(SEED, scan=3, debug=True))
    # six 60 Hz ticks of a 10 Hz head over [1079.95, 1439.95) degrees: revolution 3
    g, fired = _run_ticks(c, L, sensor, pose, 3 * 360.0 - 0.05, 10.0, 1.0 / 60.0, 6, SEED)
    assert fired == [(3, i) for i in range(sensor.n_az)]
    full_cols = _written(g, sensor)
    assert full_cols.all()
    for k in full:
        assert np.array_equal(g[k], full[k]), k


def test_rolling_shutter_tick_matches_oracle(L):
    """A moving, turning sensor on the 522k-triangle scene; the tick crosses a
    revolution boundary (two runs).  Sampled beams of the fired columns match
    the oracle; columns that did not fire keep their contents."""
    scene, sensor, pose = S.urban_64ch()
    c = _ctx(L, scene, sensor)
    pa = S.Pose(pose.p, S.quat_from_ypr(0.2, 0.01, -0.02))
    pb = S.Pose((pose.p + np.array([1.5, 0.4, 0.05])).astype(np.float32), S.quat_from_ypr(0.2 + math.radians(6.0),
                                                                                            0.015, -0.01))
    head, spin, dt = 5 * 360.0 - 100.0, 10.0, 1.0 / 20.0          # 180 degrees, 100 before and 80 after
    out = _sentinel_outputs(L, sensor.n_beams)
    out, runs = c.simulate_sweep(SEED, head, spin, dt, (pa.p, pa.q), (pb.p, pb.q), out=out)
    c.sync_check()
    g = to_np(out)
    o_runs = O.sweep_columns(sensor, *O.sweep_window(head, spin, dt))
    assert [(s, f, n) for s, f, n in runs] == [(s, lo, hi - lo) for s, lo, hi in o_runs]
    assert len(runs) == 2
    fired = np.zeros(sensor.n_az, bool)
    for s, f, n in runs:
        fired[f:f + n] = True
    assert np.array_equal(_written(g, sensor), fired)
    rng = np.random.default_rng(17)
    cols = np.flatnonzero(fired)
    beams = np.unique(np.r_[rng.choice(sensor.n_ch, 3000) * sensor.n_az + rng.choice(cols, 3000),
                            np.arange(sensor.n_ch) * sensor.n_az + cols[0],
                            np.arange(sensor.n_ch) * sensor.n_az + cols[-1]])
    o = O.simulate_sweep(scene, sensor, pa, pb, head, spin, dt, seed=SEED, beams=beams)
    rep = compare({k: v[..., beams] for k, v in g.items()}, o)
    print("[parity] sweep urban_64ch:", rep, flush=True)
    assert rep["valid"] > 1000 and rep["ambiguous"] < 0.01 * rep["n"]


def test_sweep_launch_shapes_and_lbvh_do_not_change_results(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor)
    pa = S.Pose(pose.p, S.quat_from_ypr(0.1))
    pb = S.Pose((pose.p + np.array([0.8, -0.3, 0.0])).astype(np.float32), S.quat_from_ypr(0.4, 0.02))
    ref = None
    for builder in ("ploc", "lbvh"):
        c.load(scene, builder=builder)
        for tile, lanes in ((16, 4), (1, 1), (64, 4), (4, 1), (16, 2), (2, 2)):
            c.set_tile_shape(tile)
            c.set_lanes_per_ray(lanes)
            out, _ = c.simulate_sweep(9, 30.0, 10.0, 0.07, (pa.p, pa.q), (pb.p, pb.q), debug=True)
            g = to_np(out)
            if ref is None:
                ref = g
                o = O.simulate_sweep(scene, sensor, pa, pb, 30.0, 10.0, 0.07, seed=9)
                compare({k: v[..., o["beams"]] for k, v in g.items()}, o)
            for k in ref:
                assert np.array_equal(ref[k], g[k]), (builder, tile, lanes, k)


def test_sweep_edge_cases(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor)
    pq = (pose.p, pose.q)
    out = _sentinel_outputs(L, sensor.n_beams)
    before = to_np(out)
    out, runs = c.simulate_sweep(1, 100.0, 10.0, 0.0, pq, pq, out=out)   # zero-length tick
    assert runs == []
    after = to_np(out)
    for k in before:
        assert np.array_equal(before[k], after[k], equal_nan=True), k
    out, runs = c.simulate_sweep(1, -50.0, 10.0, 0.01, pq, pq, out=out)   # [-50, -14): before revolution 0
    assert runs == []
    out, runs = c.simulate_sweep(1, -20.0, 10.0, 0.01, pq, pq, out=out)   # [-20, 16): 0.4-degree columns 0..39
    assert runs == [(0, 0, 40)]
    assert [(s, lo, hi - lo) for s, lo, hi in O.sweep_columns(sensor, -20.0, 16.0)] == runs
    out, runs = c.simulate_sweep(1, 0.0, 10.0, 0.1, pq, pq, out=out)      # exactly one revolution
    assert runs == [(0, 0, 900)]
    with pytest.raises(L.LidarError):
        c.simulate_sweep(1, 0.0, 10.0, 0.2, pq, pq)                      # 720 degrees
    with pytest.raises(L.LidarError):
        c.simulate_sweep(1, float("nan"), 10.0, 0.01, pq, pq)
    with pytest.raises(L.LidarError):
        c.simulate_sweep(1, 0.0, 10.0, 0.01, pq, (pose.p, np.array([2.0, 0, 0, 0], np.float32)))
