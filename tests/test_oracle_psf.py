"""Pins of the PSF / Strehl oracle against facts other than itself: a brute-force DFT,
Parseval, the Dirichlet-kernel closed form of a uniform square aperture, the diffraction-
limited peak, the shift theorem, piston invariance, a DM that cancels a layer, and the
Marechal approximation for small aberrations."""

import math

import numpy as np

import oracle
import synth


def _cfg(layers, lam_ref=0.5e-6):
    offs, stride = synth.layer_offsets(layers)
    for L, o in zip(layers, offs):
        L["offset"] = o
    return dict(layers=layers, layer_stride=stride, lambda_ref_m=lam_ref, dt_s=0.002)


def _layer(n, pitch, alt=0.0, w=1.0, boundary=0, vx=0.0, vy=0.0):
    return dict(nx=n, ny=n, pitch_m=pitch, alt_m=alt, vx_mps=vx, vy_mps=vy, weight=w,
                boundary=boundary)


def test_psf_frame_against_a_brute_force_dft():
    rng = np.random.default_rng(1)
    n, N = 6, 16
    A = oracle.science_pupil(6.0, 1.5, n)
    ph = rng.standard_normal((n, n))
    kap = 0.7
    got = oracle.psf_frame(ph, A, kap, N)
    E = A * np.exp(1j * kap * ph)
    want = np.zeros((N, N))
    for v in range(N):
        for u in range(N):
            acc = 0j
            for y in range(n):
                for x in range(n):
                    acc += E[y, x] * np.exp(-2j * np.pi * (u * x + v * y) / N)
            # zero frequency moved to (N/2, N/2)
            want[(v + N // 2) % N, (u + N // 2) % N] = abs(acc) ** 2 / (N * N * A.sum())
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_parseval_unit_sum_and_piston_invariance():
    rng = np.random.default_rng(2)
    A = oracle.science_pupil(8.0, 2.0, 20)
    ph = rng.standard_normal((20, 20)) * 3.0
    I = oracle.psf_frame(ph, A, 0.4, 64)
    assert abs(I.sum() - 1.0) < 1e-12
    np.testing.assert_allclose(oracle.psf_frame(ph + 2.5, A, 0.4, 64), I, atol=1e-15)
    assert abs(oracle.phase_variance(ph + 2.5, A, 0.4) - oracle.phase_variance(ph, A, 0.4)) \
        < 1e-12


def test_uniform_square_aperture_is_a_product_of_dirichlet_kernels():
    n, N = 8, 32
    I = oracle.psf_frame(np.zeros((n, n)), np.ones((n, n)), 1.0, N)
    u = np.arange(N) - N // 2
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.sin(np.pi * u * n / N) ** 2 / np.sin(np.pi * u / N) ** 2
    d[u == 0] = n * n
    want = np.outer(d, d) / (N * N * n * n)
    np.testing.assert_allclose(I, want, atol=1e-14)


def test_flat_wavefront_peak_is_the_diffraction_limit():
    A = oracle.science_pupil(8.0, 2.0, 32)
    N = 64
    I = oracle.psf_frame(np.zeros((32, 32)), A, 1.0, N)
    assert abs(I[N // 2, N // 2] - A.sum() / N ** 2) < 1e-15
    assert I.argmax() == (N // 2) * N + N // 2
    assert abs(oracle.strehl_from_psf(I, 1, A, N) - 1.0) < 1e-12


def test_tilt_moves_the_psf_by_whole_pixels():
    """A phase 2 pi k0 x / N across the pupil rolls the PSF by k0 columns (x frequency)."""
    n, N, k0 = 16, 32, 3
    A = oracle.science_pupil(4.0, 0.0, n)
    x = np.arange(n)
    tilt = np.tile(2 * np.pi * k0 * x / N, (n, 1))
    I0 = oracle.psf_frame(np.zeros((n, n)), A, 1.0, N)
    I1 = oracle.psf_frame(tilt, A, 1.0, N)
    np.testing.assert_allclose(I1, np.roll(I0, k0, axis=1), atol=1e-15)


def test_dm_cancelling_a_layer_gives_a_perfect_strehl():
    rng = np.random.default_rng(3)
    lay = [_layer(40, 0.25, alt=0.0), _layer(40, 0.25, alt=0.0, w=-1.0, boundary=1)]
    cfg = _cfg(lay)
    scr = rng.standard_normal(1600)
    buf = np.concatenate([scr, scr])
    psf, var = oracle.long_exposure(buf, cfg, [(0.0, 0.0), (1e-5, -2e-5)], [0, 3], [1e-6],
                                    [64], 8.0, 2.0, 32)
    A = oracle.science_pupil(8.0, 2.0, 32)
    for s in range(2):
        assert abs(oracle.strehl_from_psf(psf[0, s], 2, A, 64) - 1.0) < 1e-12
        assert var[0, s] < 1e-20


def test_marechal_agrees_with_the_psf_strehl_for_small_aberrations():
    rng = np.random.default_rng(4)
    n = 32
    A = oracle.science_pupil(8.0, 2.0, n)
    for sigma in (0.05, 0.1, 0.2):
        ph = rng.standard_normal((n, n)) * sigma
        I = oracle.psf_frame(ph, A, 1.0, 64)
        sr = oracle.strehl_from_psf(I, 1, A, 64)
        s2 = oracle.phase_variance(ph, A, 1.0)
        assert abs(sr - math.exp(-s2)) <= s2 ** 2 + 1e-12, (sigma, sr, math.exp(-s2))
