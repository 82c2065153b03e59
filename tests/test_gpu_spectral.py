"""GPU parity of the full-spectrum adjoint (gradient with respect to every bin
of the per-material spectral table through the interpolation at the sensor
wavelength, Section II-C / eq.4) against the FP64 oracle, and a
multi-wavelength calibration through autograd."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle.lidar_oracle as O
from lidar_inputs import scenes as S
from tests.parity import to_np

pytestmark = pytest.mark.gpu

WAVELENGTHS = (850.0, 905.0, 940.0)      # on bin 45, between bins 50 and 51, on bin 54


@pytest.fixture(scope="module")
def L():
    import paper_2208_10295_amd as lib
    return lib


@pytest.fixture(scope="module")
def c5w(L):
    """One context per wavelength (a context holds one sensor)."""
    cal = S.calibration_20mat()
    ctxs = []
    for lam in WAVELENGTHS:
        ctx = L.Context(0)
        ctx.load(cal["scene"])
        ctx.set_sensor(dataclasses.replace(cal["sensor"], wavelength_nm=lam))
        pt = cal["pose_true"]
        ctx.set_pose(pt.p, pt.q)
        ctxs.append(ctx)
    return ctxs, cal


def test_spectral_adjoint_matches_oracle(L, c5w):
    ctxs, c = c5w
    scene, pose = c["scene"], c["pose_true"]
    T_true = scene.spectra.astype(np.float64)
    T0 = (0.3 + 0.1 * np.cos(np.arange(61) / 7.0)[None, :] + 0.01 * np.arange(20)[:, None]).astype(np.float32)
    k0 = c["k_true"]
    rng = np.random.default_rng(5)
    beams = np.sort(rng.choice(c["sensor"].n_beams, 4096, replace=False))
    f32 = dict(dtype=torch.float32, device=ctxs[0].device)
    for ctx, lam in zip(ctxs, WAVELENGTHS):
        sensor = dataclasses.replace(c["sensor"], wavelength_nm=lam)
        tgt = O.simulate(scene, sensor, pose, beams=beams, rho=O.reflectance_at_wavelength(T_true, lam)[0],
                         angle_exp=k0)
        cur = O.simulate(scene, sensor, pose, beams=beams, rho=O.reflectance_at_wavelength(T0, lam)[0], angle_exp=k0)
        keep = ((tgt["valid"] == 1) & (cur["valid"] == 1) & ~tgt["ambiguous"] & ~cur["ambiguous"]
                & ~cur["grazing"] & ~cur["marginal"])
        B = beams[keep]
        N = len(B)
        assert N > 500
        z3 = np.zeros(3)
        g_T, g_k, g_pose = O.calib_grad_spectral(scene, sensor, pose, cur["tri"][keep].astype(np.int64), B, T0, k0,
                                                  z3, z3, tgt["intensity"][keep], tgt["range"][keep])
        params = dict(spectra=torch.tensor(T0, **f32), angle_exp=torch.tensor(k0, **f32),
                      pose_delta=torch.zeros(6, **f32))
        out = ctx.simulate(0, 0, debug=True, params=params)
        g = to_np(out)
        assert np.array_equal(g["tri"][B], cur["tri"][keep])
        I_t = np.zeros(sensor.n_beams, np.float32)
        R_t = np.zeros(sensor.n_beams, np.float32)
        I_t[B] = tgt["intensity"][keep]
        R_t[B] = tgt["range"][keep]
        mask = np.zeros(sensor.n_beams, np.uint8)
        mask[B] = 1
        mt = torch.tensor(mask, device=ctx.device)
        gI = (2.0 / N) * (out["intensity"] - torch.tensor(I_t, device=ctx.device)) * mt
        gR = (2.0 / N) * (out["range"] - torch.tensor(R_t, device=ctx.device)) * mt
        d_T, d_k, d_pose = ctx.backward_spectra(out["tri"], mt, gI.contiguous(), gR.contiguous(), params=params)
        d_T = d_T.cpu().numpy().astype(np.float64)
        hot = np.flatnonzero(O.spectral_weights(61, lam))
        assert np.all(d_T[:, [b for b in range(61) if b not in hot]] == 0.0)
        err = np.linalg.norm(d_T - g_T) / np.linalg.norm(g_T)
        err_k = np.linalg.norm(d_k.cpu().numpy() - g_k) / np.linalg.norm(g_k)
        print(f"[spectral] {lam:.0f} nm: bins {hot.tolist()}, d_spectra rel err {err:.3g}, d_k rel err {err_k:.3g} "
              f"(|g| {np.linalg.norm(g_T):.3g}, {N} beams)", flush=True)
        assert err < 1e-4 and err_k < 1e-4
        # the same scan through lidar_backward: d_spectra is w_b * d_rho
        d_rho, _, _ = ctx.backward(out["tri"], mt, gI.contiguous(), gR.contiguous(),
                                   params=dict(rho=torch.tensor(O.reflectance_at_wavelength(T0, lam)[0]
                                                                .astype(np.float32), **f32),
                                               angle_exp=params["angle_exp"], pose_delta=params["pose_delta"]))
        w = O.spectral_weights(61, lam)
        np.testing.assert_allclose(d_T[:, hot], np.outer(d_rho.cpu().numpy(), w[hot]), rtol=1e-5, atol=1e-9)


def test_multi_wavelength_calibration_through_autograd(L, c5w):
    """Three wavelengths in one loss: autograd's gradient is the sum of the
    three spectral adjoints, and Adam on the spectral table reduces the loss."""
    ctxs, c = c5w
    dev = ctxs[0].device
    f32 = dict(dtype=torch.float32, device=dev)
    k = torch.tensor(c["k_true"], **f32)
    pose6 = torch.zeros(6, **f32)
    with torch.no_grad():
        tgts = [L.LidarSpectralReturn.apply(cx, torch.tensor(c["scene"].spectra, **f32), k, pose6) for cx in ctxs]
    T = torch.full((20, 61), 0.3, **f32).requires_grad_(True)
    opt = torch.optim.Adam([T], lr=0.02)
    losses = []
    for it in range(30):
        opt.zero_grad()
        loss = 0.0
        ups = []
        for cx, (I_t, R_t, V_t, T_t) in zip(ctxs, tgts):
            I, R, V, Tr = L.LidarSpectralReturn.apply(cx, T, k, pose6)
            m = ((V == 1) & (V_t == 1) & (Tr == T_t)).float()
            cnt = m.sum()
            loss = loss + (((I - I_t) ** 2) * m).sum() / cnt
            ups.append((cx, Tr, m, (2.0 / cnt) * (I - I_t).detach() * m))
        loss.backward()
        if it == 0:
            want = sum(cx.backward_spectra(Tr, m.to(torch.uint8), gI.contiguous(), None,
                                           params=dict(spectra=T.detach().contiguous(), angle_exp=k,
                                                       pose_delta=pose6))[0] for cx, Tr, m, gI in ups)
            assert torch.allclose(T.grad, want, rtol=1e-5, atol=1e-10)
            touched = (T.grad != 0).any(dim=0).nonzero().flatten().tolist()
            assert set(touched) <= {45, 50, 51, 54}
        opt.step()
        with torch.no_grad():
            T.clamp_(0.0, 1.0)
        losses.append(float(loss.detach()))
    print(f"[spectral] 3-wavelength loss {losses[0]:.4g} -> {losses[-1]:.4g}", flush=True)
    assert losses[-1] < 0.3 * losses[0]


def test_spectral_params_errors(L, c5w):
    ctxs, c = c5w
    f32 = dict(dtype=torch.float32, device=ctxs[0].device)
    out = ctxs[0].simulate(0, 0, debug=True)
    with pytest.raises(L.LidarError):
        ctxs[0].simulate(0, 0, params=dict(rho=torch.ones(20, **f32), spectra=torch.ones(20, 61, **f32)))
    with pytest.raises(L.LidarError):
        ctxs[0].backward_spectra(out["tri"], out["valid"], params=dict(rho=torch.ones(20, **f32)))
