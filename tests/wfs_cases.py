"""Parity cases shared by the GPU tests: reduced sensor systems that span several kernel
tiles, ragged shapes (odd detector sizes, partly lit subapertures, odd subaperture sizes),
multi-sensor/multi-realisation batches, DM layers, and the full-size workloads."""

import math

import numpy as np

import synth
from synth.configs import ARCSEC


def _finish(cfg):
    offs, stride = synth.layer_offsets(cfg["layers"], 64)
    for L, o in zip(cfg["layers"], offs):
        L["offset"] = o
    cfg["layer_stride"] = stride
    return cfg


def ngs_case(n_sa, n_sub, N, b, D, obs=0.0, lam=0.6e-6, layers=1, n=128, pitch=None,
             photons=0.0, ro=0.0, batch=1, theta=(0.0, 0.0), wind=True):
    pitch = pitch or D / (n_sa * n_sub)
    lay = synth.configs._turbulence_layers(n_layers=layers, n=n, pitch=pitch, r0_total=0.3,
                                           h_max=8e3, wind=wind)
    sen = [synth.configs._ngs(theta_x=theta[0], theta_y=theta[1], n_sa=n_sa, n_sub=n_sub,
                              n_fft=N, bin_=b, lam=lam, photons=photons, read_noise=ro,
                              pupil_d=D, obs_d=obs)]
    return _finish(dict(name=f"ngs_{n_sa}x{n_sub}_N{N}_b{b}", layers=lay, sensors=sen,
                        batch=batch, lambda_ref_m=synth.LAMBDA_REF_M, dt_s=synth.DT_S))


def lgs_case(n_sa, n_sub, N, b, n_sensors=1, layers=2, n=128, pitch=0.25, noise=False,
             batch=1, fwhm=10e3):
    cfg = synth.small_lgs(n_sa=n_sa, n_sub=n_sub, n_fft=N, bin_=b, n_layers=layers, n=n,
                          pitch=pitch, noise=noise, n_sensors=n_sensors, batch=batch,
                          na_fwhm=fwhm)
    return cfg


def dm_case():
    """Two turbulence layers plus a zero-boundary DM grid (weight -1) smaller than the pupil
    footprint at its altitude, seen by two off-axis NGS."""
    cfg = ngs_case(8, 6, 12, 2, D=12.0, obs=3.0, layers=2, n=96, pitch=0.25, batch=2)
    cfg["layers"].append(dict(nx=11, ny=11, pitch_m=1.0, alt_m=2000.0, vx_mps=0.0, vy_mps=0.0,
                              weight=-1.0, boundary=1, r0_m=None, L0_m=None))
    s2 = dict(cfg["sensors"][0])
    s2.update(theta_x_rad=20 * ARCSEC, theta_y_rad=-10 * ARCSEC)
    cfg["sensors"].append(s2)
    return _finish(cfg)


def mixed_case(batch=2):
    """A lag-domain LGS and an FFT-path NGS (n_sub > 12) in one plan, several realisations."""
    cfg = lgs_case(6, 4, 8, 2, layers=2, n=128, pitch=0.25, noise=True, batch=batch)
    ngs = synth.configs._ngs(theta_x=15 * ARCSEC, theta_y=-20 * ARCSEC, n_sa=2, n_sub=16,
                             n_fft=32, bin_=4, lam=1.65e-6, photons=4000.0, read_noise=3.0,
                             pupil_d=cfg["sensors"][0]["pupil_d_m"],
                             obs_d=cfg["sensors"][0]["obs_d_m"])
    cfg["sensors"].append(ngs)
    return cfg


def uneven_case(fft=True, batch=3):
    """Lag-domain sensors of three subaperture sizes in one plan (an on-axis LGS of 9 x 9
    subapertures of 6 pixels, an off-axis LGS of 6 x 6 of 9 pixels, an 11 x 11 NGS of 4 pixels)
    over the same 13.5 m pupil, and optionally an FFT-path NGS (n_sub = 14); noise on."""
    cfg = lgs_case(9, 6, 12, 2, layers=2, n=128, pitch=0.25, noise=True, batch=batch)
    D = cfg["sensors"][0]["pupil_d_m"]
    obs = cfg["sensors"][0]["obs_d_m"]
    cfg["sensors"].append(synth.configs._lgs(theta_x=20 * ARCSEC, theta_y=-15 * ARCSEC, n_sa=6,
                                             n_sub=9, n_fft=18, bin_=2, photons=800.0,
                                             read_noise=2.0, pupil_d=D, obs_d=obs))
    cfg["sensors"].append(synth.configs._ngs(theta_x=-10 * ARCSEC, theta_y=25 * ARCSEC, n_sa=11,
                                             n_sub=4, n_fft=8, bin_=2, lam=0.8e-6,
                                             photons=600.0, read_noise=1.5, pupil_d=D,
                                             obs_d=obs))
    if fft:
        cfg["sensors"].append(synth.configs._ngs(theta_x=5 * ARCSEC, theta_y=5 * ARCSEC, n_sa=2,
                                                 n_sub=14, n_fft=32, bin_=4, lam=1.65e-6,
                                                 photons=4000.0, read_noise=3.0, pupil_d=D,
                                                 obs_d=obs))
    cfg["name"] = "uneven_subapertures" + ("_fft" if fft else "")
    return cfg


CASES = {
    "cfg0": lambda: synth.config0(),
    "lgs_n4_N8_b2": lambda: lgs_case(6, 4, 8, 2),
    # many layers on a small subaperture: the per-pixel gather's stencil taps outgrow the
    # lag-domain regions they share LDS with (the sensor tables must follow them)
    "lgs_n4_N8_b2_20layers": lambda: lgs_case(6, 4, 8, 2, layers=20),
    "lgs_n10_N32_b4_noise": lambda: lgs_case(12, 10, 32, 4, layers=3, n=256, noise=True),
    "lgs_n5_N10_b2_2sens_batch3": lambda: lgs_case(9, 5, 10, 2, n_sensors=2, batch=3, noise=True),
    "ngs_n6_N12_b4_oddpix": lambda: ngs_case(5, 6, 12, 4, D=6.0, obs=1.2),
    "ngs_n3_N6_b1": lambda: ngs_case(7, 3, 6, 1, D=5.0, obs=1.0, photons=300.0, ro=2.0),
    "ngs_n12_N24_b3": lambda: ngs_case(4, 12, 24, 3, D=8.0, obs=2.0, layers=3),
    "ngs_n2_N4_b2": lambda: ngs_case(6, 2, 4, 2, D=4.0, obs=0.5),
    "dm_two_ngs_batch2": dm_case,
    "fft_ngs_n14_N32_b4": lambda: ngs_case(4, 14, 32, 4, D=8.0, obs=2.0, layers=2),
    "fft_ngs_n20_N64_b2": lambda: ngs_case(3, 20, 64, 2, D=9.0, obs=2.0, layers=2, n=128),
    "fft_ngs_n64_N128_b4": lambda: ngs_case(2, 64, 128, 4, D=39.0, obs=11.0, layers=3, n=256,
                                            lam=1.65e-6, photons=5000.0, ro=3.0),
    "fft_ngs_n40_N128_b4": lambda: ngs_case(2, 40, 128, 4, D=16.0, obs=3.0, layers=2, n=128),
    "mixed_lgs_ngs_batch2": mixed_case,
    "uneven_lgs_ngs": lambda: uneven_case(fft=False),
    "uneven_lgs_ngs_fft": lambda: uneven_case(fft=True),
}


def slope_tolerance(cfg):
    """Per-slope bound: 1e-4 of the diffraction spot FWHM in binned pixels, N / (b n_sub)."""
    tol = []
    import oracle
    for s in cfg["sensors"]:
        nv = len(oracle.pupil_geometry(s)["valid"])
        t = 1e-4 * s["n_fft"] / (s["bin"] * s["n_sub"])
        tol.append(np.full(2 * nv, t))
    return np.concatenate(tol)


def layers_for(cfg, batch=None, scale=1.0, dm_seed=5):
    B = batch or cfg["batch"]
    x = synth.make_batch(cfg, range(B)).astype(np.float64)
    rng = np.random.default_rng(dm_seed)
    for L in cfg["layers"]:
        if L["weight"] < 0:  # DM actuators: a few radians
            o, n = L["offset"], L["nx"] * L["ny"]
            x[:, o:o + n] = rng.standard_normal((B, n)) * 1.5
    return (x * scale).astype(np.float32)
