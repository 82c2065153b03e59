#!/usr/bin/env python
"""Throughput of the gfx950 LiDAR simulation path on one MI355X.

Headline: rays/s of a 64-channel x 2048-azimuth scan (131,072 beams) in the
522,272-triangle procedural urban scene, one kernel launch per scan (BVH
traversal + return model + point-cloud write), inputs resident in HBM.

Also reported on the same line:
  * roofline of the trace kernel.  Node fetches and triangle-record tests per
    beam come from a CPU replay of the walk over the GPU-built tree
    (measure/walk_replay.c; equal to the GPU's counting kernel, which is
    checked here too).  The kernel is reported against the vector-ALU roof
    (algorithmic FP32 operations per launch over its mean duration from HIP
    events on its stream), and its algorithmic bytes against measured memory
    roofs at every level the bytes can come from (L1, L2, MALL, HBM), beside
    the HBM bytes the counters measured and the compulsory bytes (distinct
    nodes and records the scan touches, plus its outputs);
  * cpu_baseline: the FP64 brute-force oracle on a bounded sample of beams;
  * batched: 256 mixed sensor instances (21.4 M rays) in one persistent,
    graph-replayed launch vs 256 sequential plain launches;
  * adjoint: backward/forward time of the 20-material calibration problem and
    a 200-step calibration run;
  * sequence: 100 scans of 128 x 1024 along a trajectory in the 5.2 M-triangle
    scene;
  * BVH build time.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/sec, 64ch×2048 on 500k-tri scene; batched vs plain; backward/forward time"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes: a 4-wide node (128 B), a triangle's three vertices (36 B), the hit's material and label
# (6 B), the outputs written per beam (x, y, z, intensity, range: 20 B; label 4 B; valid 1 B)
NODE_BYTES, TRI_BYTES, HIT_BYTES, OUT_BYTES = 128, 36, 6, 25
# algorithmic FP32 ALU operations (an FMA, a min, a compare each count one): a node's four slab tests and
# their ordering, a triangle test, the return model of a beam (interpolation, cos^k, Philox, Box-Muller, eq.5)
OPS_NODE, OPS_TRI, OPS_BEAM = 72, 40, 100
# one FP32 operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the published 157.3 TFLOP/s
# counts an FMA as two and a packed pair as two more, which a data-dependent walk cannot use)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trace_scan_64x2048_522k_traffic.txt")
KERNEL_SOURCES = ("paper_2208_10295_amd/csrc/trace.hip", "paper_2208_10295_amd/csrc/lidar_device.hpp",
                  "paper_2208_10295_amd/csrc/bvh_build.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and blank lines are dropped, so that editing a comment does
    not orphan the profiles taken on unchanged kernels."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


TRAFFIC_SEQ_FILE = os.path.join(ROOT, "profiles", "trace_scan_128x1024_5m_traffic.txt")


def read_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch from the committed PMC summary, if it was taken on the current kernel source."""
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


COUNTERS_FILE = os.path.join(ROOT, "profiles", "trace_scan_64x2048_522k_counters.txt")
# wavefront VALU instructions per second one MI355X can issue: 256 CUs x 4 SIMDs x 2.4 GHz, one 64-lane
# FP32 instruction per SIMD every 4 cycles (16 lanes per cycle)
VALU_PEAK_GINST_S = 256 * 4 * 2.4 / 4


def read_counters():
    """Per-launch instruction and L2 counters from the committed PMC summary, if taken on the current source."""
    try:
        kv = {}
        for line in open(COUNTERS_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return {k: float(v) for k, v in kv.items() if k.startswith(("SQ_", "TCC_", "TCP_", "TA_"))}
    except (OSError, ValueError):
        return None


def timed_launches(fn, n, torch):
    """Run fn() n times with HIP events around each call on the current stream; returns (wall_s, [ms])."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n):
        evs[k][0].record()
        fn(k)
        evs[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def timed_region(fn, n, torch):
    """Run fn(k) for k < n back to back between two HIP events recorded on the current stream (the stream
    the kernels are launched on); returns (wall_s, mean ms per call from the events)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(n):
        fn(k)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / n


def O_weights(nbins, wavelength_nm, lambda0_nm=400.0, dlambda_nm=10.0):
    """Linear interpolation weights of a spectral table at a wavelength (for reporting only)."""
    w = [0.0] * nbins
    q = (wavelength_nm - lambda0_nm) / dlambda_nm
    if q <= 0:
        w[0] = 1.0
    elif q >= nbins - 1:
        w[-1] = 1.0
    else:
        i = int(math.floor(q))
        w[i], w[i + 1] = 1.0 - (q - i), q - i
    return w


def traversal_work(ctx, scene, sensor, pose, seed, torch):
    """Per-launch work of one scan from the CPU replay of its walk over the GPU-built tree: node fetches,
    triangle-record tests, beams with a hit, distinct nodes and records touched; the GPU counting kernel's
    totals beside it (they must agree); algorithmic and compulsory bytes."""
    import numpy as np
    from measure import walk_replay as W
    nodes, recs = ctx.debug_bvh()
    st = ctx.stats()
    r = W.replay(nodes, recs, st["root"], sensor, pose.p, pose.q, sensor.t_min,
                 W.trace_limit(sensor, scene.sigma_range), touched=True)
    _, nn, nt = ctx.simulate_counts(seed, 0)
    gn, gt = nn.cpu().numpy().view(np.uint32), nt.cpu().numpy().view(np.uint32)
    n = sensor.n_beams
    n_nodes, n_recs = int(r["node_visits"].sum(dtype=np.int64)), int(r["tri_tests"].sum(dtype=np.int64))
    n_hit = int((r["orig"] != 0xFFFFFFFF).sum())
    return {"node_fetches": n_nodes, "record_tests": n_recs, "beams_hit": n_hit,
            "node_fetches_per_ray": n_nodes / n, "record_tests_per_ray": n_recs / n,
            "replay_equals_gpu_counts": bool(np.array_equal(gn, r["node_visits"]) and
                                             np.array_equal(gt, r["tri_tests"])),
            "alg_bytes": NODE_BYTES * n_nodes + TRI_BYTES * n_recs + HIT_BYTES * n_hit + OUT_BYTES * n,
            "distinct_nodes": r["nodes_touched"], "distinct_records": r["records_touched"],
            "compulsory_bytes": 128 * r["nodes_touched"] + 48 * r["records_touched"] + OUT_BYTES * n}


def cpu_baseline(scene, sensor, pose, seed, target_s=22.0):
    import numpy as np
    import oracle.lidar_oracle as O
    rng = np.random.default_rng(12345)
    probe = np.sort(rng.choice(sensor.n_beams, 256, replace=False))
    t0 = time.perf_counter()
    O.simulate(scene, sensor, pose, seed=seed, scan=0, beams=probe)
    tp = time.perf_counter() - t0
    # the 256-beam probe carries the thread start-up, so it overstates the cost per beam: the sample takes
    # about 0.6 of target_s (10 to 15 s of CPU work)
    n = int(min(sensor.n_beams, max(256, 256 * target_s / max(tp, 1e-3))))
    beams = np.sort(rng.choice(sensor.n_beams, n, replace=False))
    t0 = time.perf_counter()
    O.simulate(scene, sensor, pose, seed=seed, scan=0, beams=beams)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "rays/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{n} seeded beams of the 64ch x 2048 scan, each tested against all {scene.n_tri} "
                      f"triangles in FP64 ({n * scene.n_tri / dt:.3e} ray-triangle tests/s, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--legs", default="all",
                    help="comma list of plain,roofs,cpu,batch,adjoint,sweep,echo,dynamic,sequence or 'all'")
    ap.add_argument("--leaf-width", type=int, default=4)
    ap.add_argument("--builder", default="ploc", choices=("ploc", "lbvh"))
    ap.add_argument("--ploc-radius", type=int, default=32)
    ap.add_argument("--collapse", default="sah", choices=("sah", "greedy"))
    ap.add_argument("--leaf-cost", type=float, default=0.0, help="leaf-step weight of the SAH collapse (0 = default)")
    ap.add_argument("--tile-az", type=int, default=0, help="64-beam tile width in azimuth steps; 0 = automatic")
    ap.add_argument("--lanes", type=int, default=4, help="lanes per ray (1, 2 or 4)")
    ap.add_argument("--xcd", type=int, default=1, help="XCD-aware block remap (0 or 1)")
    ap.add_argument("--seq-xcd", type=int, default=0,
                    help="XCD-aware block remap of the trajectory scans (0 or 1; off by default: the 128 x 1024 scans "
                         "of the 5.2M-triangle scene run 4-5 %% faster in launch order)")
    ap.add_argument("--seq-up-weight", type=float, default=0.25,
                    help="horizontal-face weight of the trajectory scene's tree (1 = surface area; the 100 scans "
                         "along the trajectory run about 10 %% faster at 0.25, at every PLOC radius tried)")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 256 MiB device copy (PMC scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding across GPUs is designed but not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    legs = ({"plain", "roofs", "cpu", "batch", "adjoint", "sweep", "echo", "dynamic", "sequence"}
            if args.legs == "all" else set(args.legs.split(",")))

    import numpy as np
    import torch
    import paper_2208_10295_amd as L
    from paper_2208_10295_amd.lidar import alloc_outputs, POINT_OUTPUTS
    from lidar_inputs import scenes as S

    seed = 2022
    scene, sensor, pose = S.urban_64ch()
    log(f"urban_64ch: {scene.n_tri} triangles, {sensor.n_beams} beams")
    ctx = L.Context(0)
    st = ctx.load(scene, args.leaf_width, builder=args.builder, ploc_radius=args.ploc_radius, collapse=args.collapse,
                  leaf_cost=args.leaf_cost)
    ctx.set_sensor(sensor)
    ctx.set_pose(pose.p, pose.q)
    ctx.set_tile_shape(args.tile_az)
    ctx.set_lanes_per_ray(args.lanes)
    ctx.set_xcd_remap(args.xcd)
    n = sensor.n_beams
    result = {"metric": METRIC, "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic"}
    result["config"] = {"workload": "plain scan: 64 channels (-25..+15 deg, denser at the horizon) x 2048 azimuth "
                                    "steps = 131,072 beams, procedural urban scene of 522,272 triangles "
                                    "(256x256 terrain cells, 400 buildings, 2,000 poles, 200 cars), 32 materials, "
                                    "905 nm, d_max 100 m, range noise 0.02 m",
                        "beams": n, "triangles": scene.n_tri, "leaf_width": st["leaf_width"], "bvh_builder": args.builder,
                        "ploc_radius": args.ploc_radius, "collapse": args.collapse,
                        "tile_az": args.tile_az or "auto (2; 16 for the batch, 8 with actors)",
                        "lanes_per_ray": args.lanes, "xcd_remap": args.xcd,
                        "bvh_nodes": st["n_nodes"], "bvh_depth": st["depth"]}
    result["bvh_build_ms"] = st["build_ms"]

    if args.copy_probe:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 268435456 bytes read, 268435456 bytes written")

    if "plain" in legs:
        out = alloc_outputs(n, POINT_OUTPUTS, ctx.device)
        scan = ctx.scan_launcher(seed, out)      # argument structs built once: one ctypes call per scan
        for w in range(args.warmup):
            scan(w)
        ctx.sync_check()
        wall, kernel_ms = timed_region(scan, args.steps, torch)
        ctx.sync_check()
        result["value"] = args.steps * n / wall
        result["ms_per_step"] = 1e3 * wall / args.steps
        result["kernel_ms"] = kernel_ms
        tv = traversal_work(ctx, scene, sensor, pose, seed, torch)
        alg_ops = OPS_NODE * tv["node_fetches"] + OPS_TRI * tv["record_tests"] + OPS_BEAM * n
        achieved = alg_ops / (kernel_ms * 1e-3) / 1e12
        traffic = read_traffic()
        secs = kernel_ms * 1e-3
        result["roofline"] = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
                              "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                              "ops_per_launch": alg_ops,
                              "ops_model": f"{OPS_NODE} per node fetch + {OPS_TRI} per triangle record + {OPS_BEAM} "
                                           "per beam (FP32 ALU operations, an FMA counting one)",
                              "hbm_frac_measured": None if traffic is None else traffic / secs / 1e9 / HBM_PEAK_GBS,
                              "hbm_frac_compulsory": tv["compulsory_bytes"] / secs / 1e9 / HBM_PEAK_GBS}
        cnt = read_counters()
        if cnt:
            # what the counters say binds: instruction issue, the texture-address path, or waiting
            ginst = cnt["SQ_INSTS_VALU"] / secs / 1e9
            result["roofline"]["counters"] = {
                "valu_insts_per_launch": cnt["SQ_INSTS_VALU"], "valu_issue_ginst_s": ginst,
                "valu_issue_frac_of_4_cycle_model": ginst / VALU_PEAK_GINST_S,
                "wave_wait_frac": cnt.get("SQ_WAIT_ANY_sum", cnt.get("SQ_WAIT_ANY", float("nan")))
                / cnt.get("SQ_WAVE_CYCLES_sum", cnt.get("SQ_WAVE_CYCLES", float("nan"))),
                "l2_hit_rate": cnt["TCC_HIT_sum"] / cnt["TCC_REQ_sum"],
                "l2_request_bytes_per_launch": 128.0 * cnt["TCC_REQ_sum"]}
        result["traversal"] = dict(tv, alg_bytes_per_ray=tv["alg_bytes"] / n, ops_per_ray=alg_ops / n,
                                   alg_gbs=tv["alg_bytes"] / secs / 1e9, kernel_source_sha256_16=kernel_source_hash())
        log(f"plain: {result['value']:.4g} rays/s, kernel {kernel_ms * 1e3:.1f} us, "
            f"{tv['node_fetches'] / n:.2f} nodes + {tv['record_tests'] / n:.2f} records per ray "
            f"(replay == GPU counts: {tv['replay_equals_gpu_counts']}), {achieved:.2f} T ALU ops/s "
            f"({achieved / ALU_PEAK_TOPS:.3f} of {ALU_PEAK_TOPS:.1f}), {tv['alg_bytes'] / secs / 1e9:.0f} GB/s "
            f"algorithmic")
        # order-preserving compaction of the scan's point cloud (detected beams only)
        comp, _, cnt = ctx.compact_launcher(out, alloc_outputs(n, POINT_OUTPUTS, ctx.device))
        for _ in range(3):
            comp()
        _, c_ms = timed_region(comp, 50, torch)
        n_pts = int(cnt.item())
        result["compact"] = {"workload": "detected points of the 64ch x 2048 scan, x/y/z/intensity/label/valid/range "
                                         "+ beam index, in beam order",
                             "us_per_scan": c_ms * 1e3, "points": n_pts, "beams": n}
        log(f"compact: {n_pts} points of {n} beams in {c_ms * 1e3:.1f} us")

    if "roofs" in legs:
        # measured memory roofs beside the published HBM peak: a 2 GiB streaming read, and 128-byte line
        # fetches by quads (one quad per beam, the scan's launch shape), each quad a dependent chain like a
        # walk, over working sets that fit one CU's L1 (16 KiB), one XCD's L2 (2 MiB), the MALL (64 MiB)
        # or only HBM (1 GiB), and over a working set the size of the scene's tree and records
        sink = torch.zeros(1, dtype=torch.float32, device=ctx.device)
        big = torch.randint(-2**31, 2**31 - 1, (512 << 20,), dtype=torch.int32, device=ctx.device)
        stream_run = L.probe_stream_launcher(big, sink)
        _, s_ms = timed_region(stream_run, 10, torch)
        stream_gbs = big.numel() * 4 / (s_ms * 1e-3) / 1e9
        blocks, steps = 2048, 32
        fetched = blocks * 64 * steps * 128
        roofs = {"hbm_stream_read_gbs": stream_gbs, "stream_bytes": 2 << 30,
                 "gather_launch": f"{blocks} blocks x 256 threads (one quad per beam of the scan), {steps} dependent "
                                  "128-B lines per quad, 32 B per lane, line indices uniform over the working set"}
        scene_ws = (int(st["node_bytes"] + st["tri_bytes"]) + 127) // 128 * 128
        for level, ws in (("l1", 16 << 10), ("l2", 2 << 20), ("mall", 64 << 20), ("hbm", 1 << 30),
                          ("scene", scene_ws)):
            run = L.probe_gather_launcher(big[: ws // 4], blocks, steps, True, sink)
            run()
            _, g_ms = timed_region(run, 20, torch)
            roofs[f"gather_{level}_gbs"] = fetched / (g_ms * 1e-3) / 1e9
            roofs[f"gather_{level}_working_set_bytes"] = ws
        del big
        if "traversal" in result:
            a = result["traversal"]["alg_gbs"]
            roofs["scan_alg_gbs"] = a
            roofs["scan_over_stream"] = a / stream_gbs
            for level in ("l1", "l2", "mall", "hbm", "scene"):
                roofs[f"scan_over_gather_{level}"] = a / roofs[f"gather_{level}_gbs"]
        result["roofs"] = roofs
        log("roofs: HBM stream read {:.0f} GB/s; dependent 128-B line gathers: L1 {:.0f}, L2 {:.0f}, MALL {:.0f}, "
            "HBM {:.0f}, scene-sized ({:.1f} MB) {:.0f} GB/s".format(
                stream_gbs, roofs["gather_l1_gbs"], roofs["gather_l2_gbs"], roofs["gather_mall_gbs"],
                roofs["gather_hbm_gbs"], scene_ws / 1e6, roofs["gather_scene_gbs"]))

    if "cpu" in legs:
        log("cpu baseline (FP64 oracle) ...")
        result["cpu_baseline"] = cpu_baseline(scene, sensor, pose, seed)
        log(f"cpu: {result['cpu_baseline']['value']:.4g} rays/s on {result['cpu_baseline']['cores']} threads")

    if "batch" in legs:
        sc_b, insts = S.batch_256()
        assert sc_b is scene
        batch = ctx.batch(insts, 256)
        nr = batch.n_rays
        bout = alloc_outputs(nr, POINT_OUTPUTS, ctx.device)
        log(f"batch: {len(insts)} instances, {nr} rays; tuning ...")
        # the tree (leaf width, and the area weight for rays near the horizontal) and the launch shape are
        # tuned on the batch itself (one lane per ray, never the best, is left out to keep the grid at 54)
        tune = batch.tune(packet_rays=(64, 256, 1024), leaf_widths=(2, 4, 8), lanes_per_ray=(2, 4), reps=5,
                          out=bout, up_weights=(1.0, 0.5, 0.25))
        for _ in range(2):
            batch.simulate(bout)
        ctx.sync_check()
        reps = 10
        wall_b, ms_b = timed_launches(lambda k: batch.simulate(bout), reps, torch)
        # the sequential baseline runs each instance as a plain scan with the plain-scan launch shape
        ctx.set_lanes_per_ray(args.lanes)
        for _ in range(1):
            batch.simulate(bout, sequential=True)
        wall_s, ms_s = timed_launches(lambda k: batch.simulate(bout, sequential=True), 3, torch)
        ctx.sync_check()
        result["batched"] = {
            "workload": "256 instances, 64 each of 16x900, 32x1800, 64x2048, 128x1024, random road poses in the "
                        "522k-triangle scene, 850/905/1550 nm, d_max U(50,200)",
            "rays": nr, "batched_rays_per_s": nr / (float(np.median(ms_b)) * 1e-3),
            "sequential_rays_per_s": nr / (float(np.median(ms_s)) * 1e-3),
            "batched_ms": float(np.median(ms_b)), "sequential_ms": float(np.median(ms_s)),
            "sequential_lanes_per_ray": args.lanes,
            "tuned_packet_rays": tune["best_packet_rays"], "tuned_leaf_width": tune["best_leaf_width"],
            "tuned_lanes_per_ray": tune["best_lanes_per_ray"],
            "tune_ms_grid_up_leaf_lanes_packet": tune["ms"].round(4).tolist(),
            "tune_up_weights": tune["up_weights"], "tuned_up_weight": tune["best_up_weight"],
            "tune_packets": [int(x) for x in tune["packet_rays"]],
            "tune_leaf_widths": [int(x) for x in tune["leaf_widths"]],
            "tune_lanes_per_ray": [int(x) for x in tune["lanes_per_ray"]]}
        result["batched"]["speedup_vs_sequential"] = (result["batched"]["batched_rays_per_s"]
                                                      / result["batched"]["sequential_rays_per_s"])
        log(f"batched {result['batched']['batched_rays_per_s']:.4g} rays/s vs sequential "
            f"{result['batched']['sequential_rays_per_s']:.4g} rays/s (tuned W={tune['best_leaf_width']}, "
            f"P={tune['best_packet_rays']}, lanes={tune['best_lanes_per_ray']}, area weight "
            f"{tune['best_up_weight']:g})")
        del batch, bout
        # the legs below run on the plain scan's tree again
        ctx.load(scene, args.leaf_width, builder=args.builder, ploc_radius=args.ploc_radius, collapse=args.collapse,
                 leaf_cost=args.leaf_cost)
        ctx.set_lanes_per_ray(args.lanes)

    if "adjoint" in legs:
        cal = S.calibration_20mat()
        cx = L.Context(0)
        cx.load(cal["scene"])
        cx.set_sensor(cal["sensor"])
        pt = cal["pose_true"]
        cx.set_pose(pt.p, pt.q)
        dev = cx.device
        f32 = dict(dtype=torch.float32, device=dev)
        rho_t = torch.tensor(cal["rho_true"], **f32)
        k_t = torch.tensor(cal["k_true"], **f32)
        zero6 = torch.zeros(6, **f32)
        labels = torch.tensor(cal["scene"].label.view(np.int32), device=dev)

        def lab(T):
            return torch.where(T >= 0, labels[T.clamp_min(0).long()], -1)
        with torch.no_grad():
            I_t, R_t, V_t, T_t = L.LidarReturn.apply(cx, rho_t, k_t, zero6)
        L_t = lab(T_t)
        rho = torch.tensor(cal["rho0"], **f32).requires_grad_(True)
        kk = torch.tensor(cal["k0"], **f32).requires_grad_(True)
        pose6 = torch.tensor(np.r_[cal["dp0"], cal["dw0"]], **f32).requires_grad_(True)
        # forward / backward timing at the initial point
        fwd_args = dict(rho=rho.detach(), angle_exp=kk.detach(), pose_delta=pose6.detach())
        fo = alloc_outputs(n, ("intensity", "range", "valid", "tri"), dev)
        for _ in range(3):
            cx.simulate(0, 0, out=fo, params=fwd_args)
        gI = torch.randn(n, **f32)
        gR = torch.randn(n, **f32)
        for _ in range(3):
            cx.backward(fo["tri"], fo["valid"], gI, gR, params=fwd_args)
        fwd = cx.scan_launcher(0, fo, params=fwd_args)
        bwd, _ = cx.backward_launcher(fo["tri"], fo["valid"], gI, gR, params=fwd_args)
        _, f_ms = timed_region(lambda k: fwd(0), 50, torch)
        _, b_ms = timed_region(bwd, 50, torch)
        # 200 steps of calibration (Adam) on rho, k, pose
        opt = torch.optim.Adam([{"params": [rho], "lr": 0.01}, {"params": [kk], "lr": 0.02},
                                {"params": [pose6], "lr": 0.002}])
        losses = []
        t0 = time.perf_counter()
        for it in range(200):
            opt.zero_grad()
            I, R, V, T = L.LidarReturn.apply(cx, rho, kk, pose6)
            m = ((V == 1) & (V_t == 1) & (lab(T) == L_t)).float()     # same object in both scans
            cnt = m.sum().clamp_min(1.0)
            loss = (((I - I_t) ** 2) * m).sum() / cnt + (((R - R_t) ** 2) * m).sum() / cnt
            loss.backward()
            opt.step()
            with torch.no_grad():
                rho.clamp_(0.0, 1.0)
                kk.clamp_(0.05, 5.0)
            losses.append(float(loss.detach()))
        torch.cuda.synchronize()
        cal_s = time.perf_counter() - t0
        used = np.zeros(20, bool)
        used[np.unique(cal["scene"].material)] = True
        rho_err = np.abs(rho.detach().cpu().numpy() - cal["rho_true"])[used]
        k_err = np.abs(kk.detach().cpu().numpy() - cal["k_true"])[used]
        pose_err = pose6.detach().cpu().numpy()
        result["adjoint"] = {
            "workload": "64ch x 2048 scan, 522k-triangle scene, 20 materials (rho, k), 6-DoF pose; loss = MSE of "
                        "intensity + MSE of range over beams valid in both scans on the same object",
            "forward_ms": f_ms, "backward_ms": b_ms, "backward_over_forward": b_ms / f_ms,
            "calibration_steps": 200, "calibration_s": cal_s, "loss_first": losses[0], "loss_last": losses[-1],
            "rho_abs_err_median": float(np.median(rho_err)), "k_abs_err_median": float(np.median(k_err)),
            "pose_delta_final": [float(x) for x in pose_err]}
        log(f"adjoint: fwd {f_ms * 1e3:.1f} us, bwd {b_ms * 1e3:.1f} us; loss {losses[0]:.4g} -> {losses[-1]:.4g}")
        del cx

        # full-spectrum adjoint: calibrate the 20 x 61 spectral tables from scans at three wavelengths
        import dataclasses
        lams = (850.0, 905.0, 940.0)
        cxs = []
        for lam in lams:
            c_ = L.Context(0)
            c_.load(cal["scene"])
            c_.set_sensor(dataclasses.replace(cal["sensor"], wavelength_nm=lam))
            c_.set_pose(pt.p, pt.q)
            cxs.append(c_)
        T_true = torch.tensor(cal["scene"].spectra, **f32)
        with torch.no_grad():
            tg = [L.LidarSpectralReturn.apply(c_, T_true, k_t, zero6) for c_ in cxs]
        Tt = torch.full((20, 61), 0.3, **f32).requires_grad_(True)
        sp_args = dict(spectra=Tt.detach(), angle_exp=k_t, pose_delta=zero6)
        cxs[1].simulate(0, 0, out=fo, params=sp_args)
        for _ in range(3):
            cxs[1].backward_spectra(fo["tri"], fo["valid"], gI, gR, params=sp_args)
        bws, _ = cxs[1].backward_launcher(fo["tri"], fo["valid"], gI, gR, params=sp_args, spectra=True)
        _, bs_ms = timed_region(bws, 50, torch)
        opt = torch.optim.Adam([Tt], lr=0.02)
        sl = []
        t0 = time.perf_counter()
        for it in range(100):
            opt.zero_grad()
            loss = 0.0
            for c_, (I_t3, _, V_t3, T_t3) in zip(cxs, tg):
                I, R, V, T = L.LidarSpectralReturn.apply(c_, Tt, k_t, zero6)
                m = ((V == 1) & (V_t3 == 1) & (T == T_t3)).float()
                loss = loss + (((I - I_t3) ** 2) * m).sum() / m.sum().clamp_min(1.0)
            loss.backward()
            opt.step()
            with torch.no_grad():
                Tt.clamp_(0.0, 1.0)
            sl.append(float(loss.detach()))
        torch.cuda.synchronize()
        sp_s = time.perf_counter() - t0
        # identifiable quantities: R_lambda(0) of every used material at the three wavelengths
        r_err = []
        for lam in lams:
            w = torch.tensor(O_weights(61, lam), **f32)
            r_err.append(((Tt.detach() - T_true) @ w).abs().cpu().numpy()[used])
        result["adjoint"]["spectral"] = {
            "workload": "same scene and pose, 20 x 61 spectral table, scans at 850 / 905 / 940 nm, intensity MSE",
            "backward_spectra_ms": bs_ms, "calibration_steps": 100, "calibration_s": sp_s,
            "loss_first": sl[0], "loss_last": sl[-1],
            "r_lambda0_abs_err_median": float(np.median(np.concatenate(r_err)))}
        log(f"spectral adjoint: bwd {bs_ms * 1e3:.1f} us; 3-wavelength loss {sl[0]:.4g} -> {sl[-1]:.4g}")
        del cxs

    if "sweep" in legs:
        # engine ticks at 60 Hz of a 10 Hz head: each tick traces the ~341 columns the head swept, with
        # rolling-shutter poses of a sensor driving at 10 m/s and turning at 10 deg/s, for 1 s of sim time
        spin, tick_hz, n_ticks = 10.0, 60.0, 60
        dt = 1.0 / tick_hz
        p0 = np.asarray(pose.p, np.float64)

        def pose_at(t):
            return ((p0 + np.array([10.0 * t, 0.0, 0.0])).astype(np.float32), S.quat_from_ypr(math.radians(10.0 * t)))
        heads = [0.0]
        for k in range(n_ticks):
            heads.append(heads[-1] + 360.0 * spin * dt)      # each tick starts where the last one ended
        ticks = [(heads[k], pose_at(k * dt), pose_at((k + 1) * dt)) for k in range(n_ticks)]
        outs = alloc_outputs(n, POINT_OUTPUTS, ctx.device)
        fired = []

        def tick(k):
            _, runs = ctx.simulate_sweep(seed, ticks[k][0], spin, dt, ticks[k][1], ticks[k][2], out=outs)
            if len(fired) < n_ticks:
                fired.append(sum(c for _, _, c in runs))
        for k in range(min(args.warmup, n_ticks)):
            tick(k)
        fired.clear()
        wall_s, ms_s = timed_region(tick, n_ticks, torch)
        ctx.sync_check()
        rays = sensor.n_ch * sum(fired)
        assert sum(fired) == n_ticks / tick_hz * spin * sensor.n_az
        gpu_s = ms_s * 1e-3 * n_ticks
        result["sweep"] = {"workload": "60 engine ticks at 60 Hz of a 10 Hz head (64ch x 2048, ~341 columns per "
                                       "tick) on the 522k-triangle scene, rolling-shutter poses at 10 m/s and "
                                       "10 deg/s yaw, 1 s of simulated time",
                           "ticks": n_ticks, "rays": rays, "rays_per_s": rays / gpu_s,
                           "tick_us_mean": ms_s * 1e3, "ticks_per_s": n_ticks / gpu_s,
                           "realtime_factor": (n_ticks / tick_hz) / gpu_s,
                           "wall_s": wall_s, "realtime_factor_wall": (n_ticks / tick_hz) / wall_s}
        log(f"sweep: {n_ticks} ticks, {ms_s * 1e3:.1f} us per tick ({rays / gpu_s:.4g} rays/s, "
            f"{(n_ticks / tick_hz) / gpu_s:.0f}x real time; host wall {wall_s * 1e3:.2f} ms)")

    if "echo" in legs:
        # divergent beams: 7 sub-rays in a 3 mrad cone per beam of the 64 x 2048 scan, up to 3 echoes
        K, E = 7, 3
        e_out = alloc_outputs(n * E, POINT_OUTPUTS, ctx.device)
        ws = None
        for _ in range(3):
            r = ctx.simulate_echoes(seed, 0, K, E, 0.003, 0.5, out=e_out, workspace=ws)
            ws = ctx._echo_workspace
        wall_e, ms_e = timed_region(lambda k: ctx.simulate_echoes(seed, k, K, E, 0.003, 0.5, out=e_out,
                                                                  workspace=ws), 50, torch)
        ctx.sync_check()
        det = [int(r["valid"][e].sum()) for e in range(E)]
        result["echo"] = {"workload": "64ch x 2048 scan of the 522k scene, 7 sub-rays per beam in a 3 mrad cone, "
                                      "echo separation 0.5 m, up to 3 echoes per beam",
                          "ms_per_scan": ms_e, "beams_per_s": n / (ms_e * 1e-3),
                          "subrays_per_s": K * n / (ms_e * 1e-3), "detected_per_echo": det}
        log(f"echo: {ms_e * 1e3:.1f} us per scan ({K * n / (ms_e * 1e-3):.4g} sub-rays/s), "
            f"detected per echo {det}")

    if "dynamic" in legs:
        # 300 moving actors (200 cars, 100 walking pedestrians) in the 522k scene: per 10 Hz frame the
        # pedestrian mesh is refit to its walking pose, the actors' top-level BVH is refit, and one scan runs
        dc = S.dynamic_actors()
        ids = [ctx.load_mesh(m) for m in dc["meshes"]]
        n_frames = 20
        frames = [ctx.actor_array(dc["actors_at"](0.1 * f)) for f in range(n_frames + 1)]
        sways = [torch.tensor(S.pedestrian_pose_vertices(dc["meshes"][3], 0.9 * f), device=ctx.device)
                 for f in range(n_frames + 1)]
        t0 = time.perf_counter()
        ctx.set_actors(dc["actors_at"](0.0))
        torch.cuda.synchronize()
        set_ms = (time.perf_counter() - t0) * 1e3
        outd = alloc_outputs(n, POINT_OUTPUTS, ctx.device)
        scan_d = ctx.scan_launcher(seed, outd)
        scan_d(0)

        def frame(f):
            ctx.refit_mesh(ids[3], sways[f + 1])
            ctx.update_actors(frames[f + 1])
            scan_d(f)
        wall_d, frame_ms = timed_region(frame, n_frames, torch)
        ctx.sync_check()
        _, scan_ms = timed_region(scan_d, 50, torch)
        n_act = int((outd["label"].view(torch.int32) >= 100000).sum())
        result["dynamic"] = {
            "workload": "522k-triangle scene + 300 actors (200 cars of 408 triangles, 100 deforming pedestrians of "
                        "304 triangles) moving at 10 Hz; per frame: pedestrian mesh refit, actor BVH refit, "
                        "64ch x 2048 scan",
            "frames": n_frames, "frame_ms_mean": frame_ms, "rays_per_s_with_updates": n / (frame_ms * 1e-3),
            "rays_per_s_with_updates_wall": n_frames * n / wall_d,
            "scan_ms_mean": scan_ms, "rays_per_s_scan": n / (scan_ms * 1e-3),
            "actors_set_ms": set_ms, "beams_on_actors_last_frame": n_act}
        log(f"dynamic: {frame_ms * 1e3:.1f} us per frame (refits + scan), scan {scan_ms * 1e3:.1f} us, "
            f"first set_actors call {set_ms:.2f} ms on the host, {n_act} beams on actors")
        ctx.clear_actors()

    if "sequence" in legs:
        sc3, s3, poses = S.urban_sequence_128ch()
        cs = L.Context(0)
        st3 = cs.load(sc3, args.leaf_width, builder=args.builder, ploc_radius=args.ploc_radius,
                      collapse=args.collapse, leaf_cost=args.leaf_cost, up_weight=args.seq_up_weight)
        cs.set_sensor(s3)
        cs.set_tile_shape(args.tile_az)
        cs.set_lanes_per_ray(args.lanes)
        cs.set_xcd_remap(args.seq_xcd)
        out3 = alloc_outputs(s3.n_beams, POINT_OUTPUTS, cs.device)
        one = cs.trajectory_launcher(seed, out3, poses)
        one(0)
        wall3, ms3 = timed_region(one, len(poses), torch)
        cs.sync_check()
        # one scan's work at the first pose, against the HBM roof: the bytes the counters measured and the
        # compulsory bytes (distinct nodes and records the scan touches, plus its outputs)
        cs.set_pose(poses[0].p, poses[0].q)
        _, k3_ms = timed_region(cs.scan_launcher(seed, out3), 50, torch)
        tv3 = traversal_work(cs, sc3, s3, poses[0], seed, torch)
        tr3 = read_traffic(TRAFFIC_SEQ_FILE)
        secs3 = k3_ms * 1e-3
        result["sequence"] = {"workload": "128ch x 1024 x 100 poses at 10 Hz, 5,224,200-triangle scene, 64 materials",
                              "xcd_remap": args.seq_xcd, "bvh_up_weight": args.seq_up_weight,
                              "rays_per_s": s3.n_beams / (ms3 * 1e-3), "ms_per_scan": ms3,
                              "rays_per_s_wall": len(poses) * s3.n_beams / wall3,
                              "bvh_build_ms": st3["build_ms"], "bvh_nodes": st3["n_nodes"],
                              "bvh_depth": st3["depth"],
                              "hbm": {"pose": 0, "kernel_ms": k3_ms, "traffic_bytes_per_scan": tr3,
                                      "hbm_frac_measured": None if tr3 is None else tr3 / secs3 / 1e9 / HBM_PEAK_GBS,
                                      "compulsory_bytes_per_scan": tv3["compulsory_bytes"],
                                      "hbm_frac_compulsory": tv3["compulsory_bytes"] / secs3 / 1e9 / HBM_PEAK_GBS,
                                      "distinct_nodes": tv3["distinct_nodes"],
                                      "distinct_records": tv3["distinct_records"],
                                      "tree_bytes": int(st3["node_bytes"] + st3["tri_bytes"]),
                                      "alg_bytes_per_scan": tv3["alg_bytes"],
                                      "alg_gbs": tv3["alg_bytes"] / secs3 / 1e9,
                                      "replay_equals_gpu_counts": tv3["replay_equals_gpu_counts"]}}
        log(f"sequence: {result['sequence']['rays_per_s']:.4g} rays/s; one scan touches "
            f"{tv3['compulsory_bytes'] / 1e6:.2f} MB (HBM fraction at {k3_ms * 1e3:.1f} us: "
            f"{result['sequence']['hbm']['hbm_frac_compulsory']:.4f})")
        # the same 100 scans (same Philox counters) as one batched launch: a recorded trajectory replayed
        # offline, where every pose is known before the first scan
        sb = cs.batch([S.Instance(s3, poses[k], seed=seed, scan=k) for k in range(len(poses))], 0)
        sbo = alloc_outputs(sb.n_rays, POINT_OUTPUTS, cs.device)
        stune = sb.tune(packet_rays=(256,), leaf_widths=(2, 4), lanes_per_ray=(2, 4), reps=3, out=sbo,
                        up_weights=(0.5, 0.25))
        sb.simulate(sbo)
        cs.sync_check()
        wall_b, ms_b = timed_launches(lambda k: sb.simulate(sbo), 5, torch)
        cs.sync_check()
        result["sequence"]["batched"] = {
            "rays_per_s": 5 * sb.n_rays / wall_b, "ms_per_trajectory": float(np.mean(ms_b)),
            "tuned_leaf_width": stune["best_leaf_width"], "tuned_lanes_per_ray": stune["best_lanes_per_ray"],
            "tuned_up_weight": stune["best_up_weight"]}
        log(f"sequence batched: {result['sequence']['batched']['rays_per_s']:.4g} rays/s "
            f"({result['sequence']['batched']['ms_per_trajectory']:.2f} ms per 100-scan trajectory)")
        del sb, sbo, cs

    if "value" not in result:
        result["value"] = None
        result["ms_per_step"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
