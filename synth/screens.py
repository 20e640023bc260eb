"""Seeded von Karman phase screens and the random reconstructor (inputs, not the method).

Screens follow the paper's description of the atmosphere module (Sec. 2.1): each layer is a
static phase screen obtained by filtering random noise in the Fourier domain with the von
Karman phase power spectrum, parameterised by r0 and L0.  The screens are periodic (they come
out of an inverse DFT), which the sensor model's periodic layer boundary relies on.
"""

import numpy as np

_SEED_BASE = (1608, 386)


def von_karman_screen(n, pitch, r0, L0, seed):
    """One n x n screen in radians at the r0 wavelength (float64).

    phi = Re( n^2 * ifft2( W * sqrt(PSD(f)) * df ) ), W = a + i b with a, b ~ N(0, 1),
    PSD(f) = 0.023 r0^(-5/3) (f^2 + L0^-2)^(-11/6), df = 1/(n*pitch), the f = 0 term zeroed.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    a = rng.standard_normal((n, n))
    b = rng.standard_normal((n, n))
    df = 1.0 / (n * pitch)
    f1 = np.fft.fftfreq(n, d=pitch)
    fx, fy = np.meshgrid(f1, f1)
    f2 = fx * fx + fy * fy
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    spec = (a + 1j * b) * np.sqrt(psd) * df
    return np.real(np.fft.ifft2(spec)) * (n * n)


def make_layers(cfg, realisation=0, dtype=np.float32, dm_values=None):
    """Flat buffer [layer_stride] for one realisation: every turbulence layer's screen placed
    at its offset.  DM grids (weight < 0) are zero unless ``dm_values`` gives their actuators
    (one flat array holding the grids back to back)."""
    buf = np.zeros(cfg["layer_stride"], dtype=np.float64)
    dm_pos = 0
    for l, L in enumerate(cfg["layers"]):
        o, n = L["offset"], L["nx"] * L["ny"]
        if L["weight"] > 0:
            assert L["nx"] == L["ny"]
            scr = von_karman_screen(L["nx"], L["pitch_m"], L["r0_m"], L["L0_m"],
                                    list(_SEED_BASE) + [realisation, l])
            buf[o:o + n] = scr.reshape(-1)
        elif dm_values is not None:
            buf[o:o + n] = dm_values[dm_pos:dm_pos + n]
            dm_pos += n
    return buf.astype(dtype)


def make_batch(cfg, realisations=None, dtype=np.float32):
    """[B][layer_stride] for realisations 0..B-1 (or the given list)."""
    if realisations is None:
        realisations = range(cfg["batch"])
    return np.stack([make_layers(cfg, r, dtype) for r in realisations])


def make_reconstructor(M, N, seed=386, dtype=np.float32):
    """R[M][N] with entries N(0,1)/sqrt(N) drawn from PCG64(seed), row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = rng.standard_normal((M, N), dtype=np.float32)
    R *= np.float32(1.0 / np.sqrt(N))
    return R.astype(dtype, copy=False)


def random_field(shape, seed, scale=1.0, dtype=np.float32):
    """Plain seeded Gaussian array (test upstream gradients, perturbations)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(shape) * scale).astype(dtype)
