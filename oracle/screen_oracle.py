"""FP64 oracle of the phase-screen generator.  TEST INFRASTRUCTURE ONLY (same rules as the
rest of this package).

Sec. 2.1: phase screens are random noise filtered in the Fourier domain with a Kolmogorov or
von Karman phase spectrum of given r0 and L0.  Reading: complex Gaussian noise W = a + i b per
Fourier sample, times sqrt(PSD) df, PSD(f) = 0.023 r0^(-5/3) (f^2 + L0^-2)^(-11/6), the f = 0
sample zeroed, and the real part of the unnormalised inverse DFT (a periodic screen).  The
normals come from Philox4x32-10 (counter: sample index k_y n + k_x, 0, stream id low/high;
key: seed low/high), Box-Muller on the first two words of each block.
"""

import numpy as np

from .philox import philox4x32_10, uniforms_from_words


def screen_normals(n, seed, stream_id):
    """(a, b) [n][n], Fourier samples in DFT order (row k_y, column k_x)."""
    idx = np.arange(n * n, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10(idx, 0, stream_id & 0xFFFFFFFF, stream_id >> 32,
                                 seed & 0xFFFFFFFF, seed >> 32)
    u0 = uniforms_from_words(w0)
    u1 = uniforms_from_words(w1)
    r = np.sqrt(-2.0 * np.log(u0))
    return (r * np.cos(2 * np.pi * u1)).reshape(n, n), (r * np.sin(2 * np.pi * u1)).reshape(n, n)


def von_karman_psd(n, pitch, r0, L0):
    """PSD(f_k) [n][n] in DFT order, the f = 0 sample zeroed (L0 = inf: Kolmogorov)."""
    f1 = np.fft.fftfreq(n, d=pitch)
    fx, fy = np.meshgrid(f1, f1)
    inv_l02 = 0.0 if np.isinf(L0) else 1.0 / (L0 * L0)
    f2 = fx * fx + fy * fy + inv_l02
    f2[0, 0] = 1.0  # replaced below
    psd = 0.023 * r0 ** (-5.0 / 3.0) * f2 ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    return psd


def screen_spectrum(n, pitch, r0, L0, seed, stream_id):
    a, b = screen_normals(n, seed, stream_id)
    df = 1.0 / (n * pitch)
    return (a + 1j * b) * np.sqrt(von_karman_psd(n, pitch, r0, L0)) * df


def phase_screen(n, pitch, r0, L0, seed, stream_id):
    """Re( n^2 ifft2(S) ): the screen [n][n] in radians."""
    S = screen_spectrum(n, pitch, r0, L0, seed, stream_id)
    return np.real(np.fft.ifft2(S)) * (n * n)
