"""Pins of the phase-screen oracle: the DFT of the screen returns the Hermitian part of the
filtered noise (so the filter, the noise and the direction of the transform are each fixed),
Philox words against the scalar known-answer implementation, normal statistics, the spectrum
against its closed form, and the phase structure function of many screens against the von
Karman / Kolmogorov law."""

import math

import numpy as np

import oracle


def test_screen_dft_is_the_hermitian_part_of_the_filtered_noise():
    n, pitch = 32, 0.1
    S = oracle.screen_spectrum(n, pitch, 0.15, 25.0, 7, 3)
    s = oracle.phase_screen(n, pitch, 0.15, 25.0, 7, 3)
    Sm = np.conj(np.roll(np.flip(S, (0, 1)), 1, (0, 1)))  # conj(S[-k])
    np.testing.assert_allclose(np.fft.fft2(s), n * n * (S + Sm) / 2, atol=1e-9 * np.abs(S).max()
                               * n * n)


def test_normals_follow_the_scalar_philox_blocks():
    n, seed, sid = 4, (5 << 32) | 17, (2 << 32) | 9
    a, b = oracle.screen_normals(n, seed, sid)
    for k in (0, 5, 15):
        w = oracle.philox4x32_10_scalar([k, 0, sid & 0xFFFFFFFF, sid >> 32],
                                        [seed & 0xFFFFFFFF, seed >> 32])
        u0 = ((w[0] >> 8) + 0.5) * 2.0 ** -24
        u1 = ((w[1] >> 8) + 0.5) * 2.0 ** -24
        r = math.sqrt(-2 * math.log(u0))
        assert abs(a.ravel()[k] - r * math.cos(2 * math.pi * u1)) < 1e-12
        assert abs(b.ravel()[k] - r * math.sin(2 * math.pi * u1)) < 1e-12


def test_normals_statistics():
    a, b = oracle.screen_normals(256, 42, 0)
    for x in (a, b):
        assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert abs((a * b).mean()) < 0.01


def test_psd_closed_form_and_zero_frequency():
    n, pitch, r0, L0 = 16, 0.2, 0.1, 20.0
    P = oracle.von_karman_psd(n, pitch, r0, L0)
    assert P[0, 0] == 0.0
    f = 3 / (n * pitch)  # sample (k_y, k_x) = (0, 3)
    assert abs(P[0, 3] - 0.023 * r0 ** (-5 / 3) * (f * f + L0 ** -2) ** (-11 / 6)) < 1e-12 * P[0, 3]
    assert P[0, 3] == P[3, 0] == P[0, n - 3]
    K = oracle.von_karman_psd(n, pitch, r0, math.inf)
    assert abs(K[0, 3] - 0.023 * r0 ** (-5 / 3) * f ** (-11 / 3)) < 1e-12 * K[0, 3]


def test_structure_function_matches_the_spectrum_and_the_kolmogorov_law():
    """D(r) = <(phi(x + r) - phi(x))^2> over 8 screens against its exact expectation for the
    discrete spectrum, 2 sum_k PSD_k df^2 (1 - cos(2 pi k r / n)), within 6 %; and against
    6.88 (r / r0)^(5/3) within [0.7, 1.0]: an FFT screen without subharmonics lacks the scales
    beyond its size, so its structure function falls short of the law (by about 23 % here)."""
    n, pitch, r0 = 256, 0.05, 0.2
    seps = (1, 2, 4)
    D = np.zeros(len(seps))
    for sid in range(8):
        s = oracle.phase_screen(n, pitch, r0, math.inf, 11, sid)
        for i, d in enumerate(seps):
            D[i] += 0.5 * (((np.roll(s, d, 1) - s) ** 2).mean()
                           + ((np.roll(s, d, 0) - s) ** 2).mean())
    D /= 8
    A2 = oracle.von_karman_psd(n, pitch, r0, math.inf) / (n * pitch) ** 2
    k = np.fft.fftfreq(n) * n
    for i, d in enumerate(seps):
        expect = 2 * (A2 * (1 - np.cos(2 * np.pi * k[None, :] * d / n))).sum()
        assert abs(D[i] / expect - 1) < 0.06, (d, D[i], expect)
        law = 6.88 * (d * pitch / r0) ** (5 / 3)
        assert 0.7 * law < D[i] < 1.0 * law, (d, D[i], law)
