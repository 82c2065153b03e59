"""CPU checks of the walk replay (measure/walk_replay.c) on hand-built trees.

The replay counts, per beam, the 4-wide nodes a walk fetches and the triangle
records it tests; the GPU's counting kernel must give the same numbers on the
GPU-built tree (checked on the GPU).  Here the counts are checked against
values worked out by hand for a tiny tree (near-first order, culling by the best
hit so far), and the replay's best hit against the FP64 brute force of the oracle
on a random soup.
"""
import numpy as np
import pytest

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from measure import walk_replay as W

EMPTY = 0xFFFFFFFF


def _leaf(first, count):
    return 0x80000000 | (first << 3) | (count - 1)


def _node(children):
    """children: up to 4 (lo, hi, ref); missing slots are empty (box at 1e30)."""
    rec = np.zeros(32, np.uint32)
    f = rec.view(np.float32)
    for s in range(4):
        base = 8 * s
        if s < len(children):
            lo, hi, ref = children[s]
        else:
            lo, hi, ref = (1e30, 1e30, 1e30), (1e30, 1e30, 1e30), EMPTY
        f[base:base + 3] = lo
        rec[base + 3] = ref
        f[base + 4:base + 7] = hi
    return rec


def _records(tris, labels=None):
    """tris: [n, 3, 3] vertices in leaf order; original index = position unless given."""
    n = len(tris)
    rec = np.zeros((n, 12), np.uint32)
    f = rec.view(np.float32)
    for k, t in enumerate(tris):
        f[k, 0:3], f[k, 4:7], f[k, 8:11] = t[0], t[1], t[2]
        rec[k, 3] = k if labels is None else labels[k]
    return rec


def _wall(x, half=3.0):
    return [np.array([[x, -half, -half], [x, half, -half], [x, half, half]], np.float32),
            np.array([[x, -half, -half], [x, half, half], [x, -half, half]], np.float32)]


def _box(tris, pad=1e-3):
    v = np.concatenate([t for t in tris])
    return tuple(v.min(axis=0) - pad), tuple(v.max(axis=0) + pad)


def _sensor(n_az, elev=(0.0,)):
    return S.Sensor(np.array(elev), n_az, d_max=100.0, noise_on=False)


def test_counts_near_first_and_culled_by_the_best_hit():
    """A child's box is tested when its parent is fetched, against the bound of that moment; a pushed
    leaf is tested when popped (its records are read whatever the bound is by then), a pushed node is
    fetched and its children are tested against the tighter bound."""
    # leaf B (wall x = 10) in slot 0, leaf C (wall x = -30) in slot 1, leaf A (wall x = 5) in slot 2
    A, B, Cw = _wall(5.0), _wall(10.0), _wall(-30.0)
    tris = B + Cw + A                                   # records: B 0-1, C 2-3, A 4-5
    recs = _records(tris)
    root = _node([(*_box(B), _leaf(0, 2)), (*_box(Cw), _leaf(2, 2)), (*_box(A), _leaf(4, 2))])
    sensor = _sensor(4)                                 # azimuths 0, 90, 180, 270 degrees at elevation 0
    q, p = np.array([1, 0, 0, 0], np.float32), np.zeros(3, np.float32)
    r = W.replay(root, recs, 0, sensor, p, q, 0.01, 100.0, touched=True)
    assert r["not_replayed"] == 0
    # +x: root; A (entry 5) before B (entry 10), both pushed leaves: 4 records, best hit A at 5
    assert (r["node_visits"][0], r["tri_tests"][0], r["leaf_visits"][0]) == (1, 4, 2)
    assert r["nodes_touched"] == 1 and r["records_touched"] == 6          # every wall seen by some beam
    assert abs(r["t"][0] - 5.0) < 1e-6 and r["orig"][0] in (4, 5)
    # +y and -y: no box is entered
    for b in (1, 3):
        assert (r["node_visits"][b], r["tri_tests"][b], r["orig"][b]) == (1, 0, EMPTY)
        assert r["t"][b] == np.float32(100.0)
    # -x: C at 30 only
    assert (r["node_visits"][2], r["tri_tests"][2]) == (1, 2) and abs(r["t"][2] - 30.0) < 1e-5
    # from x = 7.5 looking +x: B only; looking -x: A (2.5 away) then C (37.5), both leaves
    r = W.replay(root, recs, 0, _sensor(2), np.array([7.5, 0, 0], np.float32), q, 0.01, 100.0)
    assert (r["tri_tests"][0], r["tri_tests"][1]) == (2, 4)
    assert r["orig"][0] in (0, 1) and r["orig"][1] in (4, 5)
    # a trace range of 4 m: A's entry at 5 is beyond the bound 4 * 1.0000005, nothing is entered
    r = W.replay(root, recs, 0, sensor, p, q, 0.01, 4.0)
    assert (r["node_visits"][0], r["tri_tests"][0], r["orig"][0]) == (1, 0, EMPTY)


def test_two_levels_a_popped_node_sees_the_tighter_bound():
    A, B, Cw, D = _wall(5.0), _wall(10.0), _wall(15.0), _wall(-8.0)
    tris = A + B + Cw + D                                 # A 0-1, B 2-3, C 4-5, D 6-7
    recs = _records(tris)
    # node 1 holds C (slot 0) and B (slot 1); the root holds node 1, A and D
    n1 = _node([(*_box(Cw), _leaf(4, 2)), (*_box(B), _leaf(2, 2))])
    lo1, hi1 = _box(B + Cw)
    root = _node([(lo1, hi1, 1), (*_box(A), _leaf(0, 2)), (*_box(D), _leaf(6, 2))])
    nodes = np.concatenate([root, n1])
    q = np.array([1, 0, 0, 0], np.float32)
    # from the origin looking +x: A (5) first, hit; node 1 (entry 10) popped and fetched, its children B
    # (10) and C (15) lie beyond the bound 5 * 1.0000005: 2 nodes, 2 records
    r = W.replay(nodes, recs, 0, _sensor(1), np.zeros(3, np.float32), q, 0.01, 100.0)
    assert (r["node_visits"][0], r["tri_tests"][0]) == (2, 2) and r["orig"][0] in (0, 1)
    # the same without A's hit (trace limit 100, A removed by starting behind it at x = 6): node 1 is
    # entered at 4 and B at 4 is the hit; C (9 away) is pushed before the hit and then tested
    r = W.replay(nodes, recs, 0, _sensor(1), np.array([6.0, 0, 0], np.float32), q, 0.01, 100.0)
    assert (r["node_visits"][0], r["tri_tests"][0]) == (2, 4) and r["orig"][0] in (2, 3)
    # from x = 12.5: looking +x, node 1 (holds the origin) then C at 2.5; looking -x, node 1 then B at
    # 2.5, then the pushed leaves A (7.5) and D (20.5) are popped and tested
    r = W.replay(nodes, recs, 0, _sensor(2), np.array([12.5, 0, 0], np.float32), q, 0.01, 100.0)
    assert (r["node_visits"][0], r["tri_tests"][0]) == (2, 2) and r["orig"][0] in (4, 5)
    assert (r["node_visits"][1], r["tri_tests"][1]) == (2, 6) and r["orig"][1] in (2, 3)


def test_best_hit_equals_fp64_brute_force_on_a_soup():
    """On a random soup in a flat two-level tree (every leaf at most 8 records), the replay's hit equals
    the oracle's FP64 brute-force hit (same triangle, distance within 1e-5 relative) except rays the
    oracle marks ambiguous."""
    rng = np.random.default_rng(5)
    n = 64
    c = rng.uniform(-20, 20, size=(n, 3)).astype(np.float32)
    tris = [(c[k] + rng.uniform(-6, 6, size=(3, 3))).astype(np.float32) for k in range(n)]
    order = np.argsort(c[:, 0])                          # leaves: 8 consecutive triangles along x
    tris = [tris[k] for k in order]
    recs = _records(tris, labels=order.astype(np.uint32))
    leaves = [(*_box(tris[8 * L:8 * L + 8]), _leaf(8 * L, 8)) for L in range(8)]
    n1, n2 = _node(leaves[:4]), _node(leaves[4:])
    root = _node([(*_box(tris[:32]), 1), (*_box(tris[32:]), 2)])
    nodes = np.concatenate([root, n1, n2])
    sensor = S.Sensor(np.linspace(-30, 30, 31), 180, d_max=100.0, noise_on=False)
    q, p = np.array([1, 0, 0, 0], np.float32), np.array([0.5, -0.25, 0.3], np.float32)
    r = W.replay(nodes, recs, 0, sensor, p, q, 0.01, 100.0)
    verts = np.concatenate(tris).astype(np.float32)
    idx = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
    # the oracle's soup in leaf order: its triangle k is the record k, whose original index is order[k]
    scene = S.Scene(verts, idx, np.zeros(n, np.uint16), np.zeros(n, np.uint32),
                    np.full((1, 61), 0.5, np.float32), np.zeros(1, np.float32), np.ones(1, np.float32))
    o = O.simulate(scene, sensor, S.Pose(p, q))
    o_orig = np.where(o["hit"], order[np.where(o["hit"], o["tri"], 0).astype(np.int64)], EMPTY)
    ok = ~o["ambiguous"]
    assert ok.mean() > 0.95 and o["hit"].sum() > 1000
    assert np.array_equal(r["orig"][ok], o_orig[ok].astype(np.uint32))
    h = ok & o["hit"]
    assert np.all(np.abs(r["t"][h] - o["t_hit"][h]) <= 1e-5 * o["t_hit"][h])
    assert np.all(r["node_visits"] >= 1) and np.all(r["tri_tests"] <= n)
