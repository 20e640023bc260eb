"""Pins of the calibration oracle (push-pull interaction matrix, reference slopes) and of the
regularised least-squares control matrix against facts other than themselves: the exact
linearisation given by the adjoint, superposition of pokes against a planar DM surface, unseen
actuators, the SVD form of the Tikhonov solution, the pseudo-inverse and an augmented
least-squares problem, and closed-loop convergence."""

import math

import numpy as np

import oracle
import synth


def _ngs(n_sa, n_sub, N, b, D, obs=0.0, tx=0.0, ty=0.0):
    return dict(theta_x_rad=tx, theta_y_rad=ty, src_alt_m=math.inf, lambda_m=0.6e-6,
                pupil_d_m=D, obs_d_m=obs, n_sa=n_sa, n_sub=n_sub, n_fft=N, bin=b,
                valid_frac=0.5, na_fwhm_m=0.0, launch_x_m=0.0, launch_y_m=0.0, photons=0.0,
                read_noise_e=0.0)


def _lgs(n_sa, n_sub, N, b, D, obs=0.0, tx=0.0, ty=0.0):
    s = _ngs(n_sa, n_sub, N, b, D, obs=obs, tx=tx, ty=ty)
    s.update(lambda_m=589e-9, src_alt_m=90e3, na_fwhm_m=10e3, launch_x_m=0.5)
    return s


def _system(turbulence=False, wind=(0.0, 0.0)):
    """An NGS and an off-axis LGS (8 m pupil, 4 x 4 subapertures of 4 x 4 pixels) seeing a 7 x 7
    zero-boundary DM grid of pitch 2 m at the pupil (wider than the pupil: its corner actuators
    lie outside every beam), and optionally a periodic turbulence screen at 3 km moving with
    the wind (vx, vy) in m/s."""
    layers = []
    if turbulence:
        layers.append(dict(nx=48, ny=48, pitch_m=0.5, alt_m=3000.0, vx_mps=wind[0],
                           vy_mps=wind[1], weight=1.0, boundary=0))
    layers.append(dict(nx=7, ny=7, pitch_m=2.0, alt_m=0.0, vx_mps=0.0, vy_mps=0.0,
                       weight=-1.0, boundary=1))
    sensors = [_ngs(4, 4, 8, 2, D=8.0, obs=1.0),
               _lgs(4, 4, 8, 2, D=8.0, obs=1.0, tx=5e-5, ty=-3e-5)]
    offs, stride = synth.layer_offsets(layers)
    for L, o in zip(layers, offs):
        L["offset"] = o
    cfg = dict(layers=layers, sensors=sensors, batch=1, layer_stride=stride,
               lambda_ref_m=0.6e-6, dt_s=0.002)
    return cfg, offs[-1], 49


def test_push_pull_rows_equal_the_adjoint_linearisation():
    """sum_k IM[j][k] g_k = (J^T g)[actuator j]: the push-pull difference against the adjoint of
    the sensor model, at flat and on top of a turbulence screen."""
    for turbulence in (False, True):
        cfg, a0, n_act = _system(turbulence)
        rng = np.random.default_rng(3)
        base = rng.standard_normal(cfg["layer_stride"]) * 0.3 if turbulence else None
        im = oracle.interaction_matrix(cfg, a0, n_act, 1e-4, batch=8, base=base)
        x = np.zeros((1, cfg["layer_stride"])) if base is None else base[None]
        for seed in range(3):
            g = np.random.default_rng(10 + seed).standard_normal((1, im.shape[1]))
            adj = oracle.adjoint(x, cfg, 0, g)[0, a0:a0 + n_act]
            np.testing.assert_allclose(im @ g[0], adj, rtol=0, atol=1e-6 * np.abs(adj).max())


def test_unseen_actuators_give_exactly_zero_rows():
    """The outer ring of the 7 x 7 grid sits 6 m from the centre: its bilinear support ends at
    the 4 m pupil edge, so those pokes change no lit pixel.  The actuators at (+-4, +-4) m
    reach only the corner subapertures, which are not valid.  Every other actuator is seen."""
    cfg, a0, n_act = _system()
    im = oracle.interaction_matrix(cfg, a0, n_act, 0.1, batch=8)
    iy, ix = np.divmod(np.arange(n_act), 7)
    ring = (ix == 0) | (ix == 6) | (iy == 0) | (iy == 6)
    ring |= np.isin(ix, (1, 5)) & np.isin(iy, (1, 5))
    assert np.all(im[ring] == 0.0)
    assert np.all(np.abs(im[~ring]).max(axis=1) > 1e-3)


def test_pokes_superpose_to_a_planar_dm_surface():
    """A planar DM surface is reproduced exactly by bilinear interpolation, so its slopes divided
    by the (small) amplitude equal the actuator-weighted sum of the poke responses; the
    x-ramp moves the NGS spots along x only, and against the phase gradient (DM weight -1)."""
    cfg, a0, n_act = _system()
    im = oracle.interaction_matrix(cfg, a0, n_act, 1e-4, batch=8)
    xs = (np.arange(7) - 3.0) * 2.0
    ramp = np.tile(xs, (7, 1)).ravel()  # actuator value = x position (m)
    t = 1e-5
    buf = np.zeros((1, cfg["layer_stride"]))
    buf[0, a0:a0 + n_act] = t * ramp
    s, _ = oracle.forward(buf, cfg, 0, noise=False)
    lin = ramp @ im
    np.testing.assert_allclose(s[0] / t, lin, atol=1e-5 * np.abs(lin).max())
    nv = len(oracle.pupil_geometry(cfg["sensors"][0])["valid"])  # the NGS (round spots)
    sx, sy = lin[:nv], lin[nv:2 * nv]
    assert np.all(sx < -1e-2)
    assert np.abs(sy).max() <= 1e-9 * np.abs(sx).max()


def test_reference_slopes_of_a_flat_system_are_zero():
    cfg, _, _ = _system()
    assert np.abs(oracle.reference_slopes(cfg)).max() < 1e-12


def test_lse_is_the_pseudo_inverse_without_regularisation():
    rng = np.random.default_rng(1)
    im = rng.standard_normal((7, 30))
    R = oracle.regularised_lse(im, 0.0)
    np.testing.assert_allclose(R, np.linalg.pinv(im.T), atol=1e-12)
    np.testing.assert_allclose(R @ im.T, np.eye(7), atol=1e-12)


def test_tikhonov_equals_the_filtered_svd():
    rng = np.random.default_rng(2)
    im = rng.standard_normal((9, 40)) * np.linspace(0.01, 3.0, 9)[:, None]
    eps = 0.05
    R = oracle.regularised_lse(im, eps)
    U, sv, Vt = np.linalg.svd(im.T, full_matrices=False)  # D = U diag(sv) Vt
    lam = eps * (sv ** 2).sum() / 9
    ref = Vt.T @ np.diag(sv / (sv ** 2 + lam)) @ U.T
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_weighted_tikhonov_equals_augmented_least_squares():
    """R s minimises |D x - s|^2 + lambda sum_j w_j x_j^2 (solved as a stacked lstsq)."""
    rng = np.random.default_rng(4)
    im = rng.standard_normal((8, 25))
    w = np.repeat([1.0, 4.0], 4)
    eps = 0.1
    R = oracle.regularised_lse(im, eps, weights=w)
    D = im.T
    lam = eps * (D ** 2).sum() / 8
    A = np.vstack([D, np.diag(np.sqrt(lam * w))])
    for k in range(3):
        s = rng.standard_normal(25)
        x, *_ = np.linalg.lstsq(A, np.concatenate([s, np.zeros(8)]), rcond=None)
        np.testing.assert_allclose(R @ s, x, atol=1e-12)


def test_closed_loop_with_the_calibrated_reconstructor_converges():
    """Static turbulence, integrator a <- a - g R s: the slopes fall to the part of the
    measurement the DM cannot fit, (I - D R) s_0 (the sensor is close to linear at this
    turbulence strength), well below the open-loop slopes."""
    cfg, a0, n_act = _system(turbulence=True)
    rng = np.random.default_rng(6)
    x = np.zeros((1, cfg["layer_stride"]))
    x[0, :a0] = rng.standard_normal(a0) * 0.15
    im = oracle.interaction_matrix(cfg, a0, n_act, 0.05, batch=8)
    R = oracle.regularised_lse(im, 0.05)  # damps the nearly unseen modes
    s0, _ = oracle.forward(x, cfg, 0, noise=False)
    loop = dict(cfg, dm_offset=a0, gain=-0.5)
    for k in range(25):
        x, s = oracle.closed_loop_step(x, loop, R, 0, noise=False)
    s_end, _ = oracle.forward(x, cfg, 0, noise=False)
    fit = s0[0] - im.T @ (R @ s0[0])
    assert np.linalg.norm(s_end) < 0.5 * np.linalg.norm(s0)
    assert abs(np.linalg.norm(s_end) - np.linalg.norm(fit)) <= 0.05 * np.linalg.norm(s0)


def test_rows_share_one_operating_point_on_a_moving_screen():
    """Sec. 2.5: the modes are pushed through the system at one operating point.  On a base
    screen that moves with the wind, every row is taken with the screen at the calibration's
    time step, whichever call of the batched schedule holds the actuator: the matrix does not
    depend on the number of actuators per call, and equals the adjoint linearisation at that
    step."""
    cfg, a0, n_act = _system(turbulence=True, wind=(35.0, -20.0))
    base = np.random.default_rng(3).standard_normal(cfg["layer_stride"]) * 0.3
    base[a0:] = 0.0
    step = 5
    im2 = oracle.interaction_matrix(cfg, a0, n_act, 1e-4, batch=2, step=step, base=base)
    im_all = oracle.interaction_matrix(cfg, a0, n_act, 1e-4, batch=2 * n_act, step=step,
                                       base=base)
    np.testing.assert_array_equal(im2, im_all)
    g = np.random.default_rng(12).standard_normal((1, im2.shape[1]))
    adj = oracle.adjoint(base[None], cfg, step, g)[0, a0:a0 + n_act]
    np.testing.assert_allclose(im2 @ g[0], adj, rtol=0, atol=1e-6 * np.abs(adj).max())
    # the screen does move between steps: another step gives other rows
    j = 3 * 7 + 2  # an actuator near the centre, seen by both sensors
    im_late = oracle.interaction_matrix(cfg, a0 + j, 1, 1e-4, batch=2, step=step + 3, base=base)
    assert np.abs(im_late[0] - im2[j]).max() > 1e-3 * np.abs(im2[j]).max()
