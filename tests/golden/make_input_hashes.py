"""Writes input_hashes.json: the SHA-256 of every seeded synthetic workload that the tests and the benchmark
generate with lidar_inputs.scenes.

The generators are numpy PCG64 streams with fixed seeds, so their output is fixed. Pinning its hash makes a
change to a generator (a different draw order, a changed constant, a numpy that draws differently) show up
as a failing CPU test instead of as a silent change of every workload the parity tests and the benchmark
run on.

Each workload is serialised in a canonical form: arrays by dtype, shape and bytes; dataclasses field by
field; dicts by sorted key; Python scalars as int64, float64 or UTF-8. Functions inside a workload are
hashed through their values: the terrain height function on a fixed grid, the actor list of the
moving-actor workload at fixed times, and the deformed pedestrian mesh at fixed phases.

Run from the repository root: python tests/golden/make_input_hashes.py
"""
import dataclasses
import hashlib
import inspect
import json
import os
import struct
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from lidar_inputs import scenes as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "input_hashes.json")

# the workloads, by generator name; every one is called with its default (seeded) arguments
WORKLOADS = ("small_16ch", "urban_64ch", "batch_256", "calibration_20mat", "dynamic_actors",
             "urban_sequence_128ch")
ACTOR_TIMES = (0.0, 0.05, 0.1, 1.0)        # s
PED_PHASES = (0.0, 1.0, 2.5)               # rad
HEIGHT_GRID = np.linspace(-200.0, 200.0, 17)


def _feed(h, x):
    if x is None:
        h.update(b"N")
    elif isinstance(x, (bool, np.bool_)):
        h.update(b"B" + (b"\1" if x else b"\0"))
    elif isinstance(x, (int, np.integer)):
        h.update(b"I" + struct.pack("<q", int(x)))
    elif isinstance(x, (float, np.floating)):
        h.update(b"F" + struct.pack("<d", float(x)))
    elif isinstance(x, str):
        b = x.encode()
        h.update(b"S" + struct.pack("<q", len(b)) + b)
    elif isinstance(x, np.ndarray):
        a = np.ascontiguousarray(x)
        h.update(b"A" + a.dtype.str.encode() + struct.pack("<q", a.ndim) + struct.pack(f"<{a.ndim}q", *a.shape))
        h.update(a.tobytes())
    elif dataclasses.is_dataclass(x):
        h.update(b"D" + type(x).__name__.encode())
        for f in dataclasses.fields(x):
            v = getattr(x, f.name)
            h.update(f.name.encode())
            if callable(v):
                # the terrain height function, sampled on a fixed grid
                gx, gy = np.meshgrid(HEIGHT_GRID, HEIGHT_GRID)
                _feed(h, np.asarray(v(gx, gy), dtype=np.float64))
            else:
                _feed(h, v)
    elif isinstance(x, dict):
        h.update(b"M" + struct.pack("<q", len(x)))
        for k in sorted(x):
            h.update(k.encode())
            v = x[k]
            if k == "actors_at":
                for t in ACTOR_TIMES:
                    _feed(h, float(t))
                    _feed(h, v(t))
            else:
                _feed(h, v)
    elif isinstance(x, (list, tuple)):
        h.update(b"L" + struct.pack("<q", len(x)))
        for v in x:
            _feed(h, v)
    else:
        raise TypeError(f"cannot hash {type(x).__name__}")


def workload_seed(name):
    return inspect.signature(getattr(S, name)).parameters["seed"].default


def digest(name):
    h = hashlib.sha256()
    _feed(h, getattr(S, name)())
    if name == "dynamic_actors":
        ped = S.pedestrian_mesh()
        for ph in PED_PHASES:
            _feed(h, S.pedestrian_pose_vertices(ped, ph))
    return h.hexdigest()


def digests():
    return {n: {"seed": workload_seed(n), "sha256": digest(n)} for n in WORKLOADS}


if __name__ == "__main__":
    d = {"numpy": np.__version__, "workloads": digests()}
    with open(OUT, "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")
    for n, v in d["workloads"].items():
        print(f"{n:22s} seed {v['seed']:5d}  {v['sha256']}")
