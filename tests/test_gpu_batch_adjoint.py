"""GPU tests of the batched persistent form, the autotuner, the adjoint and the ABI error paths."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import compare, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


@pytest.fixture(scope="module")
def bat(L):
    scene, insts = S.batch_256()
    ctx = L.Context(0)
    ctx.load(scene)
    batch = ctx.batch(insts, 256)
    return ctx, batch, scene, insts


def test_batch_equals_sequential_and_oracle(bat):
    ctx, batch, scene, insts = bat
    assert batch.n_rays == 21_385_216 and batch.clamped     # 1550 nm instances clamp
    a = to_np(batch.simulate(debug=True))
    ctx.sync_check()
    b = to_np(batch.simulate(debug=True, sequential=True))
    ctx.sync_check()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # 1 % of the beams of every one of the 256 instances (213,852 rays) against the oracle
    rng = np.random.default_rng(4)
    tot = {}
    for k, inst in enumerate(insts):
        beams = np.sort(rng.choice(inst.sensor.n_beams, inst.sensor.n_beams // 100, replace=False))
        o = O.simulate(scene, inst.sensor, inst.pose, seed=inst.seed, scan=inst.scan, inst=int(k), beams=beams)
        off = batch.offsets[k]
        g = {key: (v[..., off + beams] if v.ndim == 2 else v[off + beams]) for key, v in a.items()}
        rep = compare(g, o)
        for key, v in rep.items():
            tot[key] = max(tot.get(key, 0), v) if key.endswith("_max_rel") else tot.get(key, 0) + v
    print(f"[parity] batch, 1 % of every instance: {tot}", flush=True)
    assert tot["n"] == sum(i.sensor.n_beams // 100 for i in insts) and tot["tri_mismatch"] == 0


def test_batch_short_stack_first_pass(bat):
    """The batched walks of one or two lanes per ray first run with a 32-entry stack (the 522k tree needs
    48), and rays that need more are traced again with the whole stack: with two lanes the automatic
    first pass, a forced 16-entry one (rays traced twice) and one pass with the whole stack all equal
    the sequential launches on all 21.4 M rays."""
    ctx, batch, _, _ = bat
    assert ctx.stats()["stack_entries"] > 32
    ref = to_np(batch.simulate(debug=True, sequential=True))
    ctx.sync_check()
    try:
        ctx.set_lanes_per_ray(2)
        for opt in (0, 16, -1):
            ctx.set_batch_stack(opt)
            got = to_np(batch.simulate(debug=True))
            ctx.sync_check()
            n = ctx.batch_restarted()
            print(f"[batch stack] option {opt}: {n} rays traced again", flush=True)
            if opt == -1:
                assert n == 0
            for k in ref:
                assert np.array_equal(ref[k], got[k]), (opt, k)
    finally:
        ctx.set_batch_stack(0)
        ctx.set_lanes_per_ray(4)


def test_batch_short_stack_every_lane_count(L):
    """A first pass of 1 or 2 stack entries (nearly every walk needs more) with 1, 2 and 4 lanes per ray:
    the second pass gives the one-pass results; with the stack capped for the whole walk (the error
    option), the second pass overflows too and sync_check reports it."""
    from paper_2208_10295_amd import _abi as A
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), n_az), pose, seed=11, scan=k) for k, n_az in
             enumerate((900, 333, 64))]
    ctx = L.Context(0)
    ctx.load(scene)
    b = ctx.batch(insts, 64)
    ctx.set_batch_stack(-1)
    ref = to_np(b.simulate(debug=True))
    ctx.sync_check()
    for lanes in (1, 2, 4):
        ctx.set_lanes_per_ray(lanes)
        for opt in (1, 2):
            ctx.set_batch_stack(opt)
            got = to_np(b.simulate(debug=True))
            ctx.sync_check()
            assert ctx.batch_restarted() > 0, (lanes, opt)
            for k in ref:
                assert np.array_equal(ref[k], got[k]), (lanes, opt, k)
    ctx.set_stack_cap(1)
    b.simulate(debug=True)
    with pytest.raises(L.LidarError) as e:
        ctx.sync_check()
    assert e.value.status == A.ERR_STACK_OVERFLOW
    ctx.set_stack_cap(0)
    for bad in (-2, 97):
        with pytest.raises(L.LidarError):
            ctx.set_batch_stack(bad)


def test_batch_may_outlive_its_context(L):
    """Destroying a context detaches its batches: a batch destroyed afterwards frees only itself and leaves
    no pending HIP error behind (the next kernel launch of another library still succeeds), and a detached
    batch is refused by the calls of another context."""
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), 64), pose, seed=1)]
    ctx = L.Context(0)
    ctx.load(scene)
    b = ctx.batch(insts, 64)
    b.simulate()
    ctx.sync_check()
    ctx.close()
    other = L.Context(0)
    other.load(scene)
    from paper_2208_10295_amd import _abi as A
    from paper_2208_10295_amd.lidar import alloc_outputs, outputs_struct, POINT_OUTPUTS
    o = outputs_struct(alloc_outputs(b.n_rays, POINT_OUTPUTS, other.device))
    assert A.lib.lidar_simulate_batch(other.h, b.h, C.byref(o), None) == A.ERR_INVALID_ARG
    b.close()
    t = torch.arange(1024, device="cuda", dtype=torch.float32)
    assert float((t * 2).sum().item()) == 1023.0 * 1024.0
    torch.cuda.synchronize()
    other.close()


def test_batch_graph_replays_are_identical(bat):
    ctx, batch, _, _ = bat
    from paper_2208_10295_amd.lidar import alloc_outputs, POINT_OUTPUTS
    out = alloc_outputs(batch.n_rays, POINT_OUTPUTS, ctx.device)
    ref = None
    for r in range(4):
        batch.simulate(out)
        torch.cuda.synchronize()
        cur = {k: v.clone() for k, v in out.items()}
        # unrelated eager work between replays
        out["x"].fill_(-1.0)
        out["label"].zero_()
        torch.cuda.synchronize()
        if ref is None:
            ref = cur
        for k in ref:
            assert torch.equal(ref[k], cur[k]), (r, k)


def test_batch_packet_sizes_identical(L):
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), n_az, wavelength_nm=wl, d_max=dm), pose, seed=9, scan=1)
             for n_az, wl, dm in ((900, 905.0, 100.0), (333, 850.0, 60.0), (64, 1000.0, 150.0))]
    ctx = L.Context(0)
    ctx.load(scene)
    ref = None
    for pk in (64, 128, 1024):
        for lanes in (1, 2, 4):
            ctx.set_lanes_per_ray(lanes)
            b = ctx.batch(insts, pk)
            g = to_np(b.simulate(debug=True))
            if ref is None:
                ref = g
            for k in ref:
                assert np.array_equal(ref[k], g[k]), (pk, lanes, k)
    for k, inst in enumerate(insts):
        o = O.simulate(scene, inst.sensor, inst.pose, seed=9, scan=1, inst=k)
        off = b.offsets[k]
        sl = slice(off, off + inst.sensor.n_beams)
        compare({key: (v[..., sl]) for key, v in ref.items()}, o)


def test_tuner_picks_a_candidate_and_keeps_results(L):
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), 900), pose, seed=3) for _ in range(4)]
    ctx = L.Context(0)
    ctx.load(scene)
    b = ctx.batch(insts, 64)
    before = to_np(b.simulate(debug=True))
    res = b.tune(packet_rays=(64, 256), leaf_widths=(1, 4), lanes_per_ray=(1, 2, 4), reps=3)
    assert res["best_packet_rays"] in (64, 256) and res["best_leaf_width"] in (1, 4)
    assert res["best_lanes_per_ray"] in (1, 2, 4) and res["ms"].shape == (2, 3, 2)
    assert np.all(res["ms"] > 0)
    assert ctx.stats()["leaf_width"] == res["best_leaf_width"]
    after = to_np(b.simulate(debug=True))
    for k in before:
        assert np.array_equal(before[k], after[k]), k


def test_tuner_area_weights(L):
    """With candidate area weights the grid gains a leading weight axis, the chosen weight is a candidate,
    the outputs are those of the untuned batch (the tree changes, the first hits do not), and a weight
    outside 1/128..255/128 is refused."""
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), 900), pose, seed=5, scan=k) for k in range(3)]
    ctx = L.Context(0)
    ctx.load(scene)
    b = ctx.batch(insts, 64)
    before = to_np(b.simulate(debug=True))
    res = b.tune(packet_rays=(64, 256), leaf_widths=(2, 4), lanes_per_ray=(2, 4), reps=2,
                 up_weights=(1.0, 0.25, 1 / 128))
    assert res["ms"].shape == (3, 2, 2, 2) and np.all(res["ms"] > 0)
    assert res["best_up_weight"] in (1.0, 0.25, 1 / 128)
    assert res["best_ms"] == pytest.approx(float(res["ms"].min()))
    after = to_np(b.simulate(debug=True))
    ctx.sync_check()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    for bad in ((0.0,), (2.0,), (float("nan"),), (1.0,) * 65):
        with pytest.raises(L.LidarError):
            b.tune(packet_rays=(64,), leaf_widths=(2,), lanes_per_ray=(2,), reps=1, up_weights=bad)


def test_batch_recaptures_after_scene_and_material_changes(L):
    """A batch's captured graph holds the scene and material tables by value: after a new scene (another
    leaf width, moved and relabelled geometry, a new buffer), new materials (more of them, so the table
    is reallocated, and a larger range noise, which lengthens the traceable range) or a new stack cap,
    the next call captures again; the batch equals the plain launches and a batch made afresh."""
    scene, sensor, pose = S.small_16ch()
    insts = [S.Instance(S.Sensor(S.elev_table(16), n_az, wavelength_nm=wl, d_max=dm), pose, seed=9, scan=1)
             for n_az, wl, dm in ((900, 905.0, 100.0), (333, 850.0, 60.0))]
    ctx = L.Context(0)
    ctx.load(scene, leaf_width=4)
    b = ctx.batch(insts, 64)

    def check(tag):
        got = to_np(b.simulate(debug=True))
        seq = to_np(b.simulate(debug=True, sequential=True))
        fresh = to_np(ctx.batch(insts, 64).simulate(debug=True))
        ctx.sync_check()
        for k in got:
            assert np.array_equal(got[k], seq[k]), (tag, k)
            assert np.array_equal(got[k], fresh[k]), (tag, k)
        return got

    first = check("initial")
    moved = S.Scene((scene.vertices.astype(np.float64) + [0.37, -0.21, 0.0]).astype(np.float32), scene.indices,
                    scene.material, scene.label + 1000, scene.spectra, scene.sigma_range, scene.angle_exp)
    ctx.load(moved, leaf_width=2)
    second = check("new scene")
    assert not np.array_equal(first["label"], second["label"])
    assert np.all(second["label"][second["valid"] == 1] > 1000)
    more = np.concatenate([moved.spectra * 0.5, moved.spectra[:3]], axis=0)
    ctx.set_materials(more, np.full(len(more), 0.3, np.float32))
    third = check("new materials")
    assert not np.array_equal(second["intensity"], third["intensity"])
    # the stack cap changes the scene descriptor the graph holds (a cap of 3 overflows: reported, then
    # lifting it restores the results)
    ctx.set_stack_cap(3)
    b.simulate(debug=True)
    with pytest.raises(L.LidarError):
        ctx.sync_check()
    ctx.set_stack_cap(0)
    fourth = check("stack cap lifted")
    for k in third:
        assert np.array_equal(third[k], fourth[k]), k


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cal(L):
    cal = S.calibration_20mat()
    ctx = L.Context(0)
    ctx.load(cal["scene"])
    ctx.set_sensor(cal["sensor"])
    pt = cal["pose_true"]
    ctx.set_pose(pt.p, pt.q)
    return ctx, cal


def test_adjoint_matches_oracle_gradient(L, cal):
    ctx, c = cal
    scene, sensor, pose = c["scene"], c["sensor"], c["pose_true"]
    dev = ctx.device
    rho0 = c["rho0"] + 0.02 * np.arange(20, dtype=np.float32) / 20
    k0 = c["k0"] + 0.2 * np.sin(np.arange(20, dtype=np.float32))
    pose0 = np.r_[c["dp0"], c["dw0"]].astype(np.float32)
    rng = np.random.default_rng(21)
    beams = np.sort(rng.choice(sensor.n_beams, 4096, replace=False))
    # target scan from the hidden parameters (oracle)
    tgt = O.simulate(scene, sensor, pose, beams=beams, rho=c["rho_true"], angle_exp=c["k_true"])
    # current scan (oracle) at the initial parameters
    R0 = O.so3_exp(pose0[3:].astype(np.float64)) @ O.rotation_from_quat(pose.q)
    p0 = pose.p.astype(np.float64) + pose0[:3].astype(np.float64)
    cur = O.simulate(scene, sensor, pose, beams=beams, rho=rho0, angle_exp=k0, R=R0, p=p0)
    keep = ((tgt["valid"] == 1) & (cur["valid"] == 1) & ~tgt["ambiguous"] & ~cur["ambiguous"]
            & ~cur["grazing"] & ~cur["marginal"])
    B = beams[keep]
    N = len(B)
    assert N > 500
    g_rho, g_k, g_pose = O.calib_grad(scene, sensor, pose, cur["tri"][keep].astype(np.int64), B, rho0, k0,
                                      pose0[:3], pose0[3:], tgt["intensity"][keep], tgt["range"][keep])
    # GPU: forward with the same parameters, backward with dL/dI, dL/drange of the same loss on B
    f32 = dict(dtype=torch.float32, device=dev)
    params = dict(rho=torch.tensor(rho0, **f32), angle_exp=torch.tensor(k0, **f32),
                  pose_delta=torch.tensor(pose0, **f32))
    out = ctx.simulate(0, 0, debug=True, params=params)
    g = to_np(out)
    assert np.array_equal(g["tri"][B], cur["tri"][keep])
    I_t = np.zeros(sensor.n_beams, np.float32)
    R_t = np.zeros(sensor.n_beams, np.float32)
    I_t[B] = tgt["intensity"][keep]
    R_t[B] = tgt["range"][keep]
    mask = np.zeros(sensor.n_beams, np.uint8)
    mask[B] = 1
    mt = torch.tensor(mask, device=dev)
    gI = (2.0 / N) * (out["intensity"] - torch.tensor(I_t, device=dev)) * mt
    gR = (2.0 / N) * (out["range"] - torch.tensor(R_t, device=dev)) * mt
    d_rho, d_k, d_pose = ctx.backward(out["tri"], mt, gI.contiguous(), gR.contiguous(), params=params)
    d_rho, d_k, d_pose = (t.cpu().numpy().astype(np.float64) for t in (d_rho, d_k, d_pose))
    for name, gg, oo in (("rho", d_rho, g_rho), ("k", d_k, g_k), ("p", d_pose[:3], g_pose[:3]),
                         ("w", d_pose[3:], g_pose[3:])):
        err = np.linalg.norm(gg - oo) / np.linalg.norm(oo)
        print(f"[adjoint] {name}: rel err {err:.3g} (|g| {np.linalg.norm(oo):.3g})", flush=True)
        assert err < 1e-4, name


def test_adjoint_with_intensity_noise_clamp_matches_oracle(L):
    """With intensity noise the forward's intensity is max(0, R_lambda + sigma_I z_I): the GPU gradient
    (clamped beams read from the forward's intensity output) against the oracle's analytic gradient with
    the same z_I (itself pinned by central differences of the clamped loss), range noise on too."""
    import dataclasses
    c = S.calibration_20mat()
    scene, pose = c["scene"], c["pose_true"]
    sig_i, seed = 0.2, 515
    sensor = dataclasses.replace(c["sensor"], noise_on=True, sigma_intensity=sig_i)
    ctx = L.Context(0)
    ctx.load(scene)
    ctx.set_sensor(sensor)
    ctx.set_pose(pose.p, pose.q)
    dev = ctx.device
    rho0 = c["rho0"] + 0.02 * np.arange(20, dtype=np.float32) / 20
    k0 = c["k0"] + 0.2 * np.sin(np.arange(20, dtype=np.float32))
    pose0 = np.r_[c["dp0"], c["dw0"]].astype(np.float32)
    rng = np.random.default_rng(22)
    beams = np.sort(rng.choice(sensor.n_beams, 4096, replace=False))
    tgt = O.simulate(scene, sensor, pose, seed=seed, beams=beams, rho=c["rho_true"], angle_exp=c["k_true"])
    R0 = O.so3_exp(pose0[3:].astype(np.float64)) @ O.rotation_from_quat(pose.q)
    p0 = pose.p.astype(np.float64) + pose0[:3].astype(np.float64)
    cur = O.simulate(scene, sensor, pose, seed=seed, beams=beams, rho=rho0, angle_exp=k0, R=R0, p=p0)
    _, z_i = O.beam_normals(seed, 0, 0, beams)
    pre = cur["r_lambda"] + np.float64(np.float32(sig_i)) * z_i
    keep = ((tgt["valid"] == 1) & (cur["valid"] == 1) & ~tgt["ambiguous"] & ~cur["ambiguous"]
            & ~cur["grazing"] & ~cur["marginal"] & (np.abs(pre) > 1e-5))
    B = beams[keep]
    N = len(B)
    assert N > 500 and 0.1 < np.mean(pre[keep] <= 0) < 0.9
    g_rho, g_k, g_pose = O.calib_grad(scene, sensor, pose, cur["tri"][keep].astype(np.int64), B, rho0, k0,
                                      pose0[:3], pose0[3:], tgt["intensity"][keep], tgt["t_hit"][keep],
                                      sig_i=float(np.float32(sig_i)), z_i=z_i[keep])
    f32 = dict(dtype=torch.float32, device=dev)
    params = dict(rho=torch.tensor(rho0, **f32), angle_exp=torch.tensor(k0, **f32),
                  pose_delta=torch.tensor(pose0, **f32))
    out = ctx.simulate(seed, 0, debug=True, params=params)
    g = to_np(out)
    assert np.array_equal(g["tri"][B], cur["tri"][keep])
    assert np.array_equal(g["intensity"][B] == 0, pre[keep] <= 0)
    I_t = np.zeros(sensor.n_beams, np.float32)
    R_t = np.zeros(sensor.n_beams, np.float32)
    I_t[B] = tgt["intensity"][keep]
    R_t[B] = tgt["range"][keep]          # the same range noise as the forward's: it cancels in R - R*
    mask = np.zeros(sensor.n_beams, np.uint8)
    mask[B] = 1
    mt = torch.tensor(mask, device=dev)
    gI = ((2.0 / N) * (out["intensity"] - torch.tensor(I_t, device=dev)) * mt).contiguous()
    gR = ((2.0 / N) * (out["range"] - torch.tensor(R_t, device=dev)) * mt).contiguous()
    with pytest.raises(L.LidarError) as e:
        ctx.backward(out["tri"], mt, gI, gR, params=params)       # the clamped beams are needed
    assert e.value.status == L._abi.ERR_NO_FORWARD_STATE
    d_rho, d_k, d_pose = ctx.backward(out["tri"], mt, gI, gR, params=params, intensity=out["intensity"])
    d_rho, d_k, d_pose = (t.cpu().numpy().astype(np.float64) for t in (d_rho, d_k, d_pose))
    for name, gg, oo in (("rho", d_rho, g_rho), ("k", d_k, g_k), ("p", d_pose[:3], g_pose[:3]),
                         ("w", d_pose[3:], g_pose[3:])):
        err = np.linalg.norm(gg - oo) / np.linalg.norm(oo)
        print(f"[adjoint clamp] {name}: rel err {err:.3g} (|g| {np.linalg.norm(oo):.3g})", flush=True)
        assert err < 1e-4, name
    # autograd saves the forward's intensity and gives the same gradient
    rho = torch.tensor(rho0, **f32).requires_grad_(True)
    kk = torch.tensor(k0, **f32).requires_grad_(True)
    p6 = torch.tensor(pose0, **f32).requires_grad_(True)
    I, R, V, T = L.LidarReturn.apply(ctx, rho, kk, p6, seed, 0)
    loss = ((I - torch.tensor(I_t, device=dev)) ** 2 * mt).sum() / N + ((R - torch.tensor(R_t, device=dev)) ** 2 * mt).sum() / N
    loss.backward()
    assert np.allclose(rho.grad.cpu().numpy(), d_rho, rtol=1e-5, atol=1e-9)
    assert np.allclose(p6.grad.cpu().numpy(), d_pose, rtol=1e-5, atol=1e-9)


def test_autograd_function_and_descent(L, cal):
    ctx, c = cal
    dev = ctx.device
    f32 = dict(dtype=torch.float32, device=dev)
    labels = torch.tensor(c["scene"].label.view(np.int32), device=dev)

    def lab(T):
        return torch.where(T >= 0, labels[T.clamp_min(0).long()], -1)
    with torch.no_grad():
        I_t, R_t, V_t, T_t = L.LidarReturn.apply(ctx, torch.tensor(c["rho_true"], **f32),
                                                 torch.tensor(c["k_true"], **f32), torch.zeros(6, **f32))
    L_t = lab(T_t)
    rho = torch.tensor(c["rho0"], **f32).requires_grad_(True)
    kk = torch.tensor(c["k0"], **f32).requires_grad_(True)
    pose6 = torch.tensor(np.r_[c["dp0"], c["dw0"]], **f32).requires_grad_(True)
    opt = torch.optim.Adam([{"params": [rho], "lr": 0.01}, {"params": [kk], "lr": 0.02},
                            {"params": [pose6], "lr": 0.002}])
    losses = []
    for it in range(40):
        opt.zero_grad()
        I, R, V, T = L.LidarReturn.apply(ctx, rho, kk, pose6)
        # beams seen in both scans on the same object
        m = ((V == 1) & (V_t == 1) & (lab(T) == L_t)).float()
        cnt = m.sum()
        loss = (((I - I_t) ** 2) * m).sum() / cnt + (((R - R_t) ** 2) * m).sum() / cnt
        loss.backward()
        if it == 0:
            # autograd's gradient is the library's backward of the same upstream gradients
            gI = (2.0 / cnt) * (I - I_t).detach() * m
            gR = (2.0 / cnt) * (R - R_t).detach() * m
            d_rho, d_k, d_pose = ctx.backward(T, V, gI.contiguous(), gR.contiguous(),
                                              params=dict(rho=rho.detach(), angle_exp=kk.detach(),
                                                          pose_delta=pose6.detach()))
            assert torch.allclose(rho.grad, d_rho, rtol=1e-5, atol=1e-12)
            assert torch.allclose(kk.grad, d_k, rtol=1e-5, atol=1e-12)
            assert torch.allclose(pose6.grad, d_pose, rtol=1e-5, atol=1e-12)
        opt.step()
        losses.append(float(loss.detach()))
    print(f"[adjoint] loss {losses[0]:.4g} -> {losses[-1]:.4g} (min {min(losses):.4g})", flush=True)
    assert losses[-1] < losses[0] and min(losses) < 0.8 * losses[0]


def test_backward_is_deterministic(L, cal):
    ctx, c = cal
    out = ctx.simulate(0, 0, debug=True)
    g = torch.randn(ctx.n_beams, device=ctx.device)
    r1 = ctx.backward(out["tri"], out["valid"], g, g)
    r2 = ctx.backward(out["tri"], out["valid"], g, g)
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)


# ----------------------------------------------------------------------------
# ABI error paths (forced from the host)
# ----------------------------------------------------------------------------
def test_error_paths(L):
    from paper_2208_10295_amd import _abi as A
    lib = A.lib
    scene, sensor, pose = S.small_16ch()
    ctx = L.Context(0)
    h = ctx.h
    # nothing loaded yet
    o = A.Outputs()
    assert lib.lidar_simulate(h, 0, 0, C.byref(o), None) == A.ERR_NOT_READY
    # bad leaf width / workspace too small
    d, keep = ctx._scene_desc(scene.vertices, scene.indices, scene.material, scene.label, 4)
    pb, sb = C.c_uint64(), C.c_uint64()
    assert lib.lidar_scene_bytes(C.byref(d), C.byref(pb), C.byref(sb)) == A.OK
    buf = torch.empty(pb.value + sb.value + 512, dtype=torch.uint8, device=ctx.device)
    p_ptr = buf.data_ptr()
    s_ptr = (p_ptr + pb.value + 255) // 256 * 256
    assert lib.lidar_scene_load(h, C.byref(d), p_ptr, pb.value - 256, s_ptr, sb.value, None) == \
        A.ERR_WORKSPACE_TOO_SMALL
    d.leaf_width = 9
    assert lib.lidar_scene_load(h, C.byref(d), p_ptr, pb.value, s_ptr, sb.value, None) == A.ERR_INVALID_ARG
    d.leaf_width = 4
    assert lib.lidar_scene_load(h, C.byref(d), p_ptr + 4, pb.value, s_ptr, sb.value, None) == A.ERR_INVALID_ARG
    # an index out of range is caught on the device
    bad = scene.indices.copy()
    bad[7, 1] = len(scene.vertices) + 5
    with pytest.raises(L.LidarError) as e:
        ctx.load_scene(scene.vertices, bad, scene.material, scene.label)
    assert e.value.status == A.ERR_INVALID_ARG
    ctx.load(scene)
    # a material id beyond the table
    ctx.set_materials(scene.spectra[:2], scene.sigma_range[:2])
    ctx.set_sensor(sensor)
    ctx.set_pose(pose.p, pose.q)
    with pytest.raises(L.LidarError):
        ctx.simulate(0, 0)
    ctx.set_materials(scene.spectra, scene.sigma_range)
    # non-unit / NaN quaternion, NaN elevation
    with pytest.raises(L.LidarError):
        ctx.set_pose(pose.p, [1.0, 0.1, 0.0, 0.0])
    with pytest.raises(L.LidarError):
        ctx.set_pose([np.nan, 0, 0], [1.0, 0.0, 0.0, 0.0])
    with pytest.raises(L.LidarError):
        ctx.set_sensor(S.Sensor(np.array([0.0, np.nan]), 10))
    # empty, oversized and inconsistent sensors are refused before anything is traced
    for bad in (S.Sensor(np.zeros(0), 10), S.Sensor(np.zeros(4), 0), S.Sensor(np.zeros(4097), 10),
                S.Sensor(np.zeros(4096), 1 << 20), S.Sensor(np.array([91.0]), 10),
                S.Sensor(np.zeros(2), 10, fov_h_deg=0.0), S.Sensor(np.zeros(2), 10, fov_h_deg=361.0),
                S.Sensor(np.zeros(2), 10, d_max=0.0), S.Sensor(np.zeros(2), 10, t_min=100.0, d_max=100.0),
                S.Sensor(np.zeros(2), 10, sigma_intensity=-1.0)):
        with pytest.raises(L.LidarError) as e:
            ctx.set_sensor(bad)
        assert e.value.status == A.ERR_INVALID_ARG
    # backward without forward state
    assert lib.lidar_backward(h, None, None, None, None, None, None, None, None, None, None) == A.ERR_NO_FORWARD_STATE
    ctx.simulate(0, 0)
    ctx.sync_check()
