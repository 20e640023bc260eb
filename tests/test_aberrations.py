"""Telescope aberrations (Sec. 2.3: additive phase maps, static or as a Zernike time series):
pins of the Zernike input generator, and (GPU) a vibration time series written into an
aberration layer by recon_apply, driving the sensors, against the oracle."""

import math

import numpy as np
import pytest

import oracle
import synth
from synth.zernike import noll_to_nm, zernike, zernike_grid


def test_zernike_closed_forms_and_noll_order():
    x, y = 0.3, -0.4
    r, t = math.hypot(x, y), math.atan2(y, x)
    assert abs(zernike(1, np.array(x), np.array(y)) - 1.0) < 1e-15
    assert abs(zernike(2, np.array(x), np.array(y)) - 2 * r * math.cos(t)) < 1e-14
    assert abs(zernike(3, np.array(x), np.array(y)) - 2 * r * math.sin(t)) < 1e-14
    assert abs(zernike(4, np.array(x), np.array(y)) - math.sqrt(3) * (2 * r * r - 1)) < 1e-14
    assert abs(zernike(11, np.array(x), np.array(y))
               - math.sqrt(5) * (6 * r ** 4 - 6 * r * r + 1)) < 1e-14
    assert [noll_to_nm(j) for j in (5, 6, 7, 8)] == [(2, -2), (2, 2), (3, -1), (3, 1)]


def test_zernike_modes_are_orthonormal_on_the_disk():
    n = 801
    Z = zernike_grid(20, n, 2.0 / n, 1.0, first=1)
    inside = np.abs(Z[0]) > 0
    G = (Z[:, inside] @ Z[:, inside].T) / inside.sum()
    np.testing.assert_allclose(G, np.eye(20), atol=3e-3)


def _aberration_system():
    from wfs_cases import ngs_case
    cfg = ngs_case(8, 6, 12, 2, D=12.0, obs=3.0, layers=1, n=96, pitch=0.25, batch=1)
    nx = 52  # 13 m of map at the pupil pitch: the 12 m pupil and a margin
    cfg["layers"].append(dict(nx=nx, ny=nx, pitch_m=0.25, alt_m=0.0, vx_mps=0.0, vy_mps=0.0,
                              weight=1.0, boundary=1, r0_m=None, L0_m=None))
    offs, stride = synth.layer_offsets(cfg["layers"], 64)
    for L, o in zip(cfg["layers"], offs):
        L["offset"] = o
    cfg["layer_stride"] = stride
    return cfg, offs[-1], nx


@pytest.mark.gpu
def test_zernike_vibration_series_through_recon_apply_matches_oracle():
    import torch
    import paper_1608_00386_amd as W
    from wfs_cases import slope_tolerance
    cfg, o, nx = _aberration_system()
    Z = zernike_grid(14, nx, 0.25, 6.0)  # tip .. Z15 over the 12 m pupil
    x = np.zeros((1, cfg["layer_stride"]))
    L0 = cfg["layers"][0]
    scr = synth.von_karman_screen(L0["nx"], L0["pitch_m"], L0["r0_m"], L0["L0_m"], [1608, 7])
    x[0, L0["offset"]:L0["offset"] + L0["nx"] * L0["ny"]] = scr.ravel() * 0.3
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    Rt = torch.from_numpy(np.ascontiguousarray(Z.T).astype(np.float32)).cuda()  # [pixels][modes]
    plan = W.Plan(cfg)
    amp = np.linspace(0.5, 0.1, 14)
    for k in (0, 3, 11):
        c = amp * np.sin(2 * np.pi * (k + 1) * np.arange(1, 15) / 40.0)  # vibrations
        ct = torch.from_numpy(c[None].astype(np.float32)).cuda()
        W.recon_apply(Rt, ct, xt[:, o:o + nx * nx], alpha=1.0, beta=0.0,
                      ldc=cfg["layer_stride"])
        s, _ = plan.forward(xt, step=k)
        ref = x.copy()
        ref[0, o:o + nx * nx] = Z.T @ c.astype(np.float32).astype(np.float64)
        s_ref, _ = oracle.forward(ref, cfg, k, noise=False)
        err = np.abs(s.cpu().numpy()[0] - s_ref[0]) / slope_tolerance(cfg)
        assert err.max() <= 1.0, (k, err.max())
