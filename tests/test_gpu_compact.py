"""GPU order-preserving compaction of the point cloud (detected beams only).

The compacted cloud must equal the dense outputs indexed by the valid mask,
bit for bit and in beam order, and its beam set must equal the oracle's point
cloud except on the rays the oracle marks ambiguous or marginal.  All calls go
through the C ABI.
"""
import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import to_np

pytestmark = pytest.mark.gpu

SEED = 0x1234_5678_9ABC


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


@pytest.fixture(scope="module")
def c1(L):
    scene, sensor, pose = S.small_16ch()
    return _ctx(L, scene, sensor, pose)


def _ctx(L, scene, sensor, pose):
    c = L.Context(0)
    c.load(scene)
    c.set_sensor(sensor)
    c.set_pose(pose.p, pose.q)
    return c


def _check_against_dense(dense_np, pts, idx, cnt):
    keep = np.flatnonzero(dense_np["valid"] != 0)
    assert cnt == len(keep)
    np.testing.assert_array_equal(idx.cpu().numpy().view(np.uint32), keep.astype(np.uint32))
    g = to_np(pts)
    for k, a in dense_np.items():
        want = a[..., keep]
        assert g[k].dtype == want.dtype and g[k].shape == want.shape, k
        assert np.array_equal(np.ascontiguousarray(g[k]).view(np.uint8), np.ascontiguousarray(want).view(np.uint8)), k


def test_16ch_point_cloud_matches_dense_and_oracle(L):
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    dense = c.simulate(SEED, 2, debug=True)
    pts, idx, cnt = c.compact(dense)
    c.sync_check()
    dn = to_np(dense)
    _check_against_dense(dn, pts, idx, cnt)
    print(f"[compact] small_16ch: {cnt} of {sensor.n_beams} beams detected", flush=True)
    # against the oracle's point cloud: same beams except rays it marks ambiguous or marginal
    o = O.simulate(scene, sensor, pose, seed=SEED, scan=2)
    pc = O.point_cloud(o)
    unsure = np.flatnonzero(o["ambiguous"] | o["marginal"])
    g_beams = set(idx.cpu().numpy().tolist()) - set(unsure.tolist())
    o_beams = set(pc["beam"].tolist()) - set(unsure.tolist())
    assert g_beams == o_beams
    assert len(unsure) < 0.01 * sensor.n_beams
    # per point: range within 1e-5 relative, label exact (grazing hits excluded for the range)
    common = np.array(sorted(g_beams))
    gi = np.searchsorted(idx.cpu().numpy(), common)
    oi = np.searchsorted(pc["beam"], common)
    lab = pts["label"].cpu().numpy().view(np.uint32)[gi]
    np.testing.assert_array_equal(lab, pc["label"][oi].astype(np.uint32))
    ok = ~o["grazing"][common]
    rg = pts["range"].cpu().numpy()[gi][ok]
    assert np.all(np.abs(rg - pc["range"][oi][ok]) <= 1e-5 * pc["range"][oi][ok])


@pytest.mark.parametrize("n", [0, 1, 63, 64, 257, 1000, 262144, 300001, 524288, 600001])
@pytest.mark.parametrize("density", [0.0, 0.37, 1.0])
def test_synthetic_dense_arrays_ragged_sizes(c1, n, density):
    """Any dense arrays (not only simulated ones): empty, single, ragged tails; up to 2,048 blocks of 256
    beams (524,288) each block sums the counts before it, above that (600,001 beams = 2,344 blocks, three
    1024-block chunks) a separate prefix-sum launch runs."""
    c = c1
    g = torch.Generator().manual_seed(n * 7 + int(density * 100))
    dev = c.device
    dense = {
        "valid": (torch.rand(n, generator=g) < density).to(torch.uint8).to(dev),
        "x": torch.randn(n, generator=g).to(dev),
        "label": torch.randint(-2**31, 2**31 - 1, (n,), generator=g, dtype=torch.int32).to(dev),
        "material": torch.randint(-2**15, 2**15 - 1, (n,), generator=g, dtype=torch.int16).to(dev),
        "normal": torch.randn(3, n, generator=g).to(dev),
    }
    pts, idx, cnt = c.compact(dense)
    c.sync_check()
    _check_against_dense(to_np(dense), pts, idx, cnt)


def test_subset_of_fields_and_missing_source(L, c1):
    c = c1
    dense = c.simulate(SEED, 0)
    pts, idx, cnt = c.compact(dense, names=("x", "y", "z", "label"))
    assert set(pts) == {"x", "y", "z", "label"}
    keep = np.flatnonzero(dense["valid"].cpu().numpy())
    for k in pts:
        assert np.array_equal(pts[k].cpu().numpy(), dense[k].cpu().numpy()[keep]), k
    with pytest.raises(L.LidarError):
        c.compact({k: dense[k] for k in ("valid", "x")}, names=("x", "tri"),
                  out={"x": torch.empty_like(dense["x"]), "tri": torch.empty_like(dense["label"])})
    with pytest.raises(L.LidarError):
        c.compact({"x": dense["x"], "valid": None}, names=("x",))


def test_echo_outputs_compact_per_echo_plane(L):
    """Multi-echo outputs are [echo][beam] planes: compacting all planes at once lists echo 0's
    points, then echo 1's, each in beam order."""
    scene, sensor, pose = S.small_16ch()
    c = _ctx(L, scene, sensor, pose)
    r = c.simulate_echoes(SEED, 0, 7, 2, 0.01, 0.5)
    dense = {k: v.reshape(-1) for k, v in r.items()}
    pts, idx, cnt = c.compact(dense)
    c.sync_check()
    _check_against_dense(to_np(dense), pts, idx, cnt)
    e1 = idx.cpu().numpy() >= sensor.n_beams
    assert np.all(np.diff(idx.cpu().numpy()) > 0) and e1.sum() == int(r["valid"][1].sum())
