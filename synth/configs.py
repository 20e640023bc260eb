"""Workload presets: telescope, guide stars, turbulence layers and deformable mirrors.

Each preset is a plain dict::

    {"name", "layers": [layer, ...], "sensors": [sensor, ...], "batch", "lambda_ref_m",
     "dt_s", "steps", "seed_noise", ...}

with ``layer`` and ``sensor`` dicts whose keys are the fields of ``wfs_layer_desc`` and
``wfs_sensor_desc`` in ``include/wfs.h`` (plus ``r0_m``/``L0_m`` for screen synthesis, which the
sensor model does not see).  The numbers restate the paper's MAORY system (six sodium laser
guide stars feeding Shack-Hartmann sensors plus three natural guide stars, Sec. 1; the
0.04875 m pupil sampling of Sec. 2; frozen-flow layers of Sec. 2.1; DMs with 1 m actuator
pitch, Sec. 2) and the readings where the paper is silent (pupil obstruction, ring radii,
wavelengths, photon counts, wind profile, layer altitudes).
"""

import math

LAMBDA_REF_M = 500e-9  # screens are radians of phase at 500 nm (the r0 wavelength)
DT_S = 1.0 / 500.0  # 500 Hz loop
ARCSEC = math.pi / (180.0 * 3600.0)
GOLDEN_DEG = 137.5

ELT_D = 39.0
ELT_OBS = 11.0
ELT_PITCH = 0.04875  # m per pupil/layer pixel (Sec. 2: 740 px at 4.875e-2 m)
LGS_ALT = 90e3
LGS_LAMBDA = 589e-9
NA_FWHM = 10e3


def _turbulence_layers(n_layers=10, n=1024, pitch=ELT_PITCH, r0_total=0.157, L0=25.0,
                       h_max=16e3, wind=True):
    """Equal-strength layers at h_l = h_max*l/(L-1); |v_l| = 5 + 25 l/(L-1) m/s at l*137.5 deg.

    The integrated r0 is split evenly in C_n^2: r0_l = r0 * L**(3/5).
    """
    r0_l = r0_total * n_layers ** 0.6
    layers = []
    for l in range(n_layers):
        frac = l / (n_layers - 1) if n_layers > 1 else 0.0
        speed = 5.0 + 25.0 * frac if wind else 0.0
        ang = math.radians(GOLDEN_DEG * l)
        layers.append(dict(nx=n, ny=n, pitch_m=pitch, alt_m=h_max * frac,
                           vx_mps=speed * math.cos(ang), vy_mps=speed * math.sin(ang),
                           weight=1.0, boundary=0, r0_m=r0_l, L0_m=L0))
    return layers


def _lgs(theta_x=0.0, theta_y=0.0, n_sa=80, n_sub=10, n_fft=32, bin_=4, photons=1000.0,
         read_noise=3.0, na_fwhm=NA_FWHM, pupil_d=ELT_D, obs_d=ELT_OBS):
    return dict(theta_x_rad=theta_x, theta_y_rad=theta_y, src_alt_m=LGS_ALT,
                lambda_m=LGS_LAMBDA, pupil_d_m=pupil_d, obs_d_m=obs_d, n_sa=n_sa, n_sub=n_sub,
                n_fft=n_fft, bin=bin_, valid_frac=0.5, na_fwhm_m=na_fwhm, launch_x_m=0.0,
                launch_y_m=0.0, photons=photons, read_noise_e=read_noise)


def _ngs(theta_x=0.0, theta_y=0.0, n_sa=2, n_sub=64, n_fft=128, bin_=4, lam=1.65e-6,
         photons=5000.0, read_noise=3.0, pupil_d=ELT_D, obs_d=ELT_OBS):
    return dict(theta_x_rad=theta_x, theta_y_rad=theta_y, src_alt_m=math.inf, lambda_m=lam,
                pupil_d_m=pupil_d, obs_d_m=obs_d, n_sa=n_sa, n_sub=n_sub, n_fft=n_fft,
                bin=bin_, valid_frac=0.5, na_fwhm_m=0.0, launch_x_m=0.0, launch_y_m=0.0,
                photons=photons, read_noise_e=read_noise)


def layer_offsets(layers, pad_to=1):
    """Element offsets of each layer inside one realisation's flat buffer, and the stride."""
    offs, o = [], 0
    for L in layers:
        offs.append(o)
        o += L["nx"] * L["ny"]
    stride = ((o + pad_to - 1) // pad_to) * pad_to
    return offs, stride


def _finish(cfg):
    offs, stride = layer_offsets(cfg["layers"], cfg.get("stride_pad", 64))
    for L, o in zip(cfg["layers"], offs):
        L["offset"] = o
    cfg["layer_stride"] = cfg.get("layer_stride", stride)
    return cfg


def config0():
    """Plain forward: one on-axis NGS, 8 m, 8x8 subaps of 8 px, 16-px FFT, 4x4 binning.

    One 256x256 layer at 0.125 m (r0 = 0.15 m, L0 = 25 m), lambda = 0.6 um, noise off.
    """
    layers = [dict(nx=256, ny=256, pitch_m=0.125, alt_m=0.0, vx_mps=0.0, vy_mps=0.0,
                   weight=1.0, boundary=0, r0_m=0.15, L0_m=25.0)]
    sensors = [_ngs(n_sa=8, n_sub=8, n_fft=16, bin_=4, lam=0.6e-6, photons=0.0,
                    read_noise=0.0, pupil_d=8.0, obs_d=0.0)]
    return _finish(dict(name="config0_ngs_8x8", layers=layers, sensors=sensors, batch=1,
                        lambda_ref_m=LAMBDA_REF_M, dt_s=DT_S, steps=1, seed_noise=42))


def config1(n_layers=10, noise=True):
    """E-ELT single on-axis LGS: 80x80 subaps of 10 px, 32-px FFT, 8x8 spots, 10 layers."""
    layers = _turbulence_layers(n_layers=n_layers)
    sensors = [_lgs(photons=1000.0 if noise else 0.0, read_noise=3.0 if noise else 0.0)]
    return _finish(dict(name="config1_lgs_80x80", layers=layers, sensors=sensors, batch=1,
                        lambda_ref_m=LAMBDA_REF_M, dt_s=DT_S, steps=100, seed_noise=42))


def _ring_sensors(noise=True, with_ngs=True):
    sensors = []
    for k in range(6):  # LGS on a 2-arcmin-diameter ring
        a = math.radians(60.0 * k)
        sensors.append(_lgs(theta_x=60 * ARCSEC * math.cos(a), theta_y=60 * ARCSEC * math.sin(a),
                            photons=1000.0 if noise else 0.0,
                            read_noise=3.0 if noise else 0.0))
    if with_ngs:
        for k in range(3):  # NGS on a 160-arcsec-diameter triangle
            a = math.radians(90.0 + 120.0 * k)
            sensors.append(_ngs(theta_x=80 * ARCSEC * math.cos(a),
                                theta_y=80 * ARCSEC * math.sin(a),
                                photons=5000.0 if noise else 0.0,
                                read_noise=3.0 if noise else 0.0))
    return sensors


def config2(batch=8):
    """Batched: 6 LGS + 3 NGS, 8 realisations, 100 frozen-flow steps at 500 Hz."""
    return _finish(dict(name="config2_batched_6lgs_3ngs", layers=_turbulence_layers(),
                        sensors=_ring_sensors(), batch=batch, lambda_ref_m=LAMBDA_REF_M,
                        dt_s=DT_S, steps=100, seed_noise=42))


def config3():
    """Adjoint: the six LGS of config 2, one realisation, noise off."""
    return _finish(dict(name="config3_adjoint_6lgs", layers=_turbulence_layers(),
                        sensors=_ring_sensors(noise=False, with_ngs=False), batch=1,
                        lambda_ref_m=LAMBDA_REF_M, dt_s=DT_S, steps=1, seed_noise=42,
                        truth_realisation=0, guess_realisation=1))


DM_GRIDS = ((40, 1.0, 0.0), (42, 1.0, 4000.0), (45, 1.06, 12700.0))
N_ACT_ROWS = 5400


def config4(batch=8):
    """Closed loop: config 2 plus three zonal DMs (0/4/12.7 km) as weight -1 layers.

    The DM actuator grids sit at the end of each realisation's buffer, contiguous, so that the
    reconstructor output rows 0..5388 land on them; the stride leaves room for all 5,400 rows.
    """
    layers = _turbulence_layers()
    for n, pitch, alt in DM_GRIDS:
        layers.append(dict(nx=n, ny=n, pitch_m=pitch, alt_m=alt, vx_mps=0.0, vy_mps=0.0,
                           weight=-1.0, boundary=1, r0_m=None, L0_m=None))
    cfg = dict(name="config4_closed_loop", layers=layers, sensors=_ring_sensors(), batch=batch,
               lambda_ref_m=LAMBDA_REF_M, dt_s=DT_S, steps=1000, seed_noise=42, gain=0.4,
               n_act_rows=N_ACT_ROWS, seed_R=386, stride_pad=1)
    offs, _ = layer_offsets(layers)
    n_turb = sum(1 for L in layers if L["weight"] > 0)
    dm_off = offs[n_turb]
    cfg["dm_offset"] = dm_off
    stride = dm_off + N_ACT_ROWS
    cfg["layer_stride"] = ((stride + 63) // 64) * 64
    return _finish(cfg)


def small_lgs(n_sa=6, n_sub=4, n_fft=8, bin_=2, n_layers=2, n=64, pitch=0.5, noise=False,
              na_fwhm=NA_FWHM, n_sensors=1, batch=1):
    """Reduced LGS system used by the parity tests: a few subaps, a few small layers."""
    D = n_sa * n_sub * pitch
    layers = _turbulence_layers(n_layers=n_layers, n=n, pitch=pitch, r0_total=0.4)
    sensors = []
    for k in range(n_sensors):
        a = math.radians(60.0 * k)
        r = 0.0 if n_sensors == 1 else 30 * ARCSEC
        sensors.append(_lgs(theta_x=r * math.cos(a), theta_y=r * math.sin(a), n_sa=n_sa,
                            n_sub=n_sub, n_fft=n_fft, bin_=bin_,
                            photons=1000.0 if noise else 0.0,
                            read_noise=3.0 if noise else 0.0, na_fwhm=na_fwhm,
                            pupil_d=D, obs_d=D * 11.0 / 39.0))
    return _finish(dict(name=f"small_lgs_{n_sa}x{n_sub}_{n_fft}", layers=layers,
                        sensors=sensors, batch=batch, lambda_ref_m=LAMBDA_REF_M, dt_s=DT_S,
                        steps=1, seed_noise=42))
