"""The seeded synthetic workloads are the ones the committed hashes were taken on.

Every parity test and the benchmark generate their inputs from lidar_inputs.scenes. Their hashes, written
by tests/golden/make_input_hashes.py, pin those inputs: a generator change fails here, on the CPU, and the
hashes are then rewritten on purpose together with the figures that depend on the inputs.
"""
import importlib.util
import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("make_input_hashes", os.path.join(GOLDEN, "make_input_hashes.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


M = _maker()
STORED = json.load(open(os.path.join(GOLDEN, "input_hashes.json")))["workloads"]


def test_every_workload_is_pinned():
    assert set(STORED) == set(M.WORKLOADS)


@pytest.mark.parametrize("name", M.WORKLOADS)
def test_workload_hash(name):
    assert M.workload_seed(name) == STORED[name]["seed"]
    assert M.digest(name) == STORED[name]["sha256"], f"{name}: generated input differs from the pinned one"


def test_hash_sees_a_one_ulp_change():
    # the canonical serialisation covers the array payloads: a one-ulp change of one vertex changes the hash
    import hashlib
    import numpy as np
    from lidar_inputs import scenes as S
    scene, sensor, pose = S.small_16ch()
    h0 = hashlib.sha256()
    M._feed(h0, scene)
    scene.vertices[7, 1] = np.nextafter(scene.vertices[7, 1], np.float32(np.inf))
    h1 = hashlib.sha256()
    M._feed(h1, scene)
    assert h0.hexdigest() != h1.hexdigest()
