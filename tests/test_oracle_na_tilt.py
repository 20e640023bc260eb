"""Pins of the oracle's time-varying multi-peak sodium profile (Sec. 2.7) and per-sensor
tip-tilt offsets (Sec. 2.3, NGS WFS mispositioning) against facts other than the oracle's own
formulas: the shift theorem (a narrow peak above the focus moves the spot by an exact number of
FFT pixels away from the launch, along x or y as the baseline points), the reduction of a
one-peak profile to the single Gaussian, superposition with normalised weights, flux
conservation, the period of the profile table, a tilt of whole FFT pixels rolling the spot
along the right axis, and central finite differences of the loss through both."""

import math

import numpy as np

import oracle
import synth

H = 90e3


def _lgs(fwhm=10e3):
    """6 x 6 subapertures of 4 x 4 pixels on a 6 m pupil, N = 16, b = 2, launched from the
    centre of subaperture (a, b) = (2, 2): subaperture (2, 5) lies 3 m along +x from the
    launch and (5, 2) 3 m along +y."""
    return dict(theta_x_rad=0.0, theta_y_rad=0.0, src_alt_m=H, lambda_m=589e-9, pupil_d_m=6.0,
                obs_d_m=0.0, n_sa=6, n_sub=4, n_fft=16, bin=2, valid_frac=0.5,
                na_fwhm_m=fwhm, launch_x_m=-0.5, launch_y_m=-0.5, photons=0.0,
                read_noise_e=0.0)


def _cfg(sensor, layers=None, profile=None):
    layers = layers or [dict(nx=32, ny=32, pitch_m=0.25, alt_m=0.0, vx_mps=0.0, vy_mps=0.0,
                             weight=1.0, boundary=0)]
    offs, stride = synth.layer_offsets(layers)
    for L, o in zip(layers, offs):
        L["offset"] = o
    cfg = dict(layers=layers, sensors=[sensor], batch=1, lambda_ref_m=sensor["lambda_m"],
               dt_s=0.002, layer_stride=stride)
    if profile is not None:
        cfg["na_profile"] = profile
    return cfg


def _index(geo, a, b):
    return int(np.nonzero((geo["valid"][:, 0] == a) & (geo["valid"][:, 1] == b))[0][0])


def _trace(cfg, x, step=0):
    tr = {}
    oracle.sensor_slopes(x, cfg, 0, step, 0, 0, noise=False, trace=tr)
    return tr


def _p_fft(sensor):
    dx = sensor["pupil_d_m"] / (sensor["n_sa"] * sensor["n_sub"])
    return sensor["lambda_m"] / (sensor["n_fft"] * dx)


def test_narrow_peak_above_focus_shifts_spot_away_from_launch():
    """A zero-width peak dh above the focus seen at baseline |b|: the spot moves by
    |b| dh / (H^2 p_fft) FFT pixels along +b.  dh chosen for exactly 3 pixels."""
    sensor = _lgs()
    dh = 3.0 * H * H * _p_fft(sensor) / 3.0  # |b| = 3 m
    x = np.random.default_rng(1).standard_normal(32 * 32) * 0.4
    base = _trace(_cfg(sensor, profile=[[(0.0, 0.0, 1.0)]]), x)
    shifted = _trace(_cfg(sensor, profile=[[(dh, 0.0, 1.0)]]), x)
    geo = base["geo"]
    ix, iy = _index(geo, 2, 5), _index(geo, 5, 2)
    # zero width and no offset: no elongation at all
    np.testing.assert_allclose(base["I_e"], base["I"], rtol=0, atol=1e-14 * base["I"].max())
    np.testing.assert_allclose(shifted["I_e"][ix], np.roll(base["I"][ix], 3, axis=1), rtol=0,
                               atol=1e-12 * base["I"].max())
    np.testing.assert_allclose(shifted["I_e"][iy], np.roll(base["I"][iy], 3, axis=0), rtol=0,
                               atol=1e-12 * base["I"].max())
    # the launch subaperture itself (|b| = 0) does not move
    i0 = _index(geo, 2, 2)
    np.testing.assert_allclose(shifted["I_e"][i0], base["I"][i0], rtol=0,
                               atol=1e-12 * base["I"].max())


def test_one_peak_profile_is_the_single_gaussian():
    sensor = _lgs(fwhm=7e3)
    geo = oracle.pupil_geometry(sensor)
    K0 = oracle.elongation_kernel(sensor, geo)
    K1 = oracle.elongation_kernel(sensor, geo, [(0.0, 7e3, 5.0)])
    np.testing.assert_allclose(K1, K0, rtol=0, atol=1e-15)


def test_peaks_superpose_with_normalised_weights_and_keep_the_flux():
    sensor = _lgs()
    x = np.random.default_rng(2).standard_normal(32 * 32) * 0.4
    p1, p2 = (1500.0, 3e3, 1.0), (-2500.0, 6e3, 1.0)
    both = _trace(_cfg(sensor, profile=[[(p1[0], p1[1], 3.0), (p2[0], p2[1], 1.0)]]), x)
    a = _trace(_cfg(sensor, profile=[[p1]]), x)
    b = _trace(_cfg(sensor, profile=[[p2]]), x)
    np.testing.assert_allclose(both["I_e"], 0.75 * a["I_e"] + 0.25 * b["I_e"], rtol=0,
                               atol=1e-13 * a["I"].max())
    np.testing.assert_allclose(both["I_e"].sum(axis=(1, 2)), both["I"].sum(axis=(1, 2)),
                               rtol=1e-12)
    # the offset peaks move the centroid of the radially elongated spots outwards on average
    s_both, _ = oracle.sensor_slopes(x, _cfg(sensor, profile=[[(4000.0, 2e3, 1.0)]]), 0, 0, 0, 0,
                                     noise=False)
    s_ref, _ = oracle.sensor_slopes(x, _cfg(sensor), 0, 0, 0, 0, noise=False)
    geo = a["geo"]
    nv = len(geo["valid"])
    c = oracle.subap_centres(sensor, geo) - np.array([sensor["launch_x_m"], sensor["launch_y_m"]])
    radial = (s_both[:nv] - s_ref[:nv]) * c[:, 0] + (s_both[nv:] - s_ref[nv:]) * c[:, 1]
    assert radial.mean() > 0


def test_profile_table_entry_follows_the_step_with_its_period():
    sensor = _lgs()
    pa, pb, pc = [(0.0, 8e3, 1.0)], [(900.0, 4e3, 2.0), (-700.0, 3e3, 1.0)], [(-300.0, 1e4, 1.0)]
    x = np.random.default_rng(3).standard_normal(32 * 32) * 0.4
    cfg3 = _cfg(sensor, profile=[pa, pb, pc])
    for step, entry in ((4, pb), (6, pa), (8, pc)):
        s3, _ = oracle.sensor_slopes(x, cfg3, 0, step, 0, 0, noise=False)
        s1, _ = oracle.sensor_slopes(x, _cfg(sensor, profile=[entry]), 0, step, 0, 0,
                                     noise=False)
        np.testing.assert_array_equal(s3, s1)
    s_other, _ = oracle.sensor_slopes(x, cfg3, 0, 7, 0, 0, noise=False)  # entry pb, not pc
    assert np.abs(s_other - s3).max() > 1e-3


def _ngs(N=16, b=2):
    return dict(theta_x_rad=0.0, theta_y_rad=0.0, src_alt_m=math.inf, lambda_m=0.6e-6,
                pupil_d_m=4.0, obs_d_m=0.0, n_sa=4, n_sub=4, n_fft=N, bin=b, valid_frac=0.5,
                na_fwhm_m=0.0, launch_x_m=0.0, launch_y_m=0.0, photons=0.0, read_noise_e=0.0)


def test_tilt_of_whole_fft_pixels_rolls_the_spot_along_its_axis():
    """A tilt of k0 FFT pixels (k0 p_fft radians) on a flat wavefront rolls every spot by k0
    along x (tilt_x) or y (tilt_y), towards larger indices for a positive tilt; with k0 a
    multiple of the binning the detector image rolls by k0 / b binned pixels."""
    x = np.zeros(32 * 32)
    flat = _trace(_cfg(_ngs()), x)
    for key, axis in (("tilt_x_rad", 2), ("tilt_y_rad", 1)):
        s = _ngs()
        s[key] = 4 * _p_fft(s)
        tr = _trace(_cfg(s), x)
        np.testing.assert_allclose(tr["I"], np.roll(flat["I"], 4, axis=axis), rtol=0,
                                   atol=1e-12 * flat["I"].max())
        np.testing.assert_allclose(tr["B"], np.roll(flat["B"], 2, axis=axis), rtol=0,
                                   atol=1e-12 * flat["B"].max())
    # a small positive tilt moves the centroid the same way
    s = _ngs()
    s["tilt_x_rad"] = 0.1 * _p_fft(s)
    sl, _ = oracle.sensor_slopes(x, _cfg(s), 0, 0, 0, 0, noise=False)
    nv = len(flat["geo"]["valid"])
    assert np.all(sl[:nv] > 0) and np.allclose(sl[nv:], 0.0, atol=1e-12)


def test_adjoint_with_profile_and_tilt_against_central_differences():
    cfg = synth.small_lgs(n_sa=4, n_sub=4, n_fft=8, bin_=2, n_layers=2, n=32, pitch=0.5,
                          n_sensors=2)
    cfg["na_profile"] = [[(600.0, 3e3, 2.0), (-900.0, 5e3, 1.0)], [(200.0, 8e3, 1.0)]]
    cfg["sensors"][0]["tilt_x_rad"] = 0.3 * _p_fft(cfg["sensors"][0])
    cfg["sensors"][1]["tilt_y_rad"] = -0.2 * _p_fft(cfg["sensors"][1])
    x0 = synth.make_layers(cfg, 1).astype(np.float64)[None] * 0.5
    target, _ = oracle.forward(synth.make_layers(cfg, 0).astype(np.float64)[None] * 0.5, cfg,
                               3, noise=False)
    for step in (2, 3):
        s0, _ = oracle.forward(x0, cfg, step, noise=False)
        g = oracle.adjoint(x0, cfg, step, 2.0 * (s0 - target))
        rng = np.random.default_rng(11 + step)
        h = 1e-4
        dirs = [rng.standard_normal(x0.shape) for _ in range(4)]
        for idx in np.argsort(-np.abs(g[0]))[:4]:
            d = np.zeros_like(x0)
            d[0, idx] = 1.0
            dirs.append(d)
        for d in dirs:
            fd = (oracle.loss(x0 + h * d, cfg, step, target)
                  - oracle.loss(x0 - h * d, cfg, step, target)) / (2 * h)
            an = float((g * d).sum())
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (step, fd, an)
