"""FP64 oracle of the PSF / Strehl module.  TEST INFRASTRUCTURE ONLY (same rules as the rest
of this package).

Sec. 2.8: PSFs are computed at a user wavelength and pixel scale (several wavelengths over a
band if wanted) for the test stars; the Strehl ratio comes either from the PSF or from the
closed-loop wavefront history through the Marechal approximation.  Readings: the residual
phase of a test star (at infinity) is the projection of the layers (DM grids with weight -1)
on the full pupil grid; the PSF is |DFT of A exp(i phase) zero-padded to N x N|^2 normalised
to unit sum per frame, fftshifted (zero frequency at (N/2, N/2)), summed over frames; the PSF
Strehl ratio is the long-exposure image at zero frequency over the diffraction-limited peak;
the Marechal Strehl ratio is exp(-<sigma^2>), sigma^2 the piston-removed variance of the
phase over the lit pupil, averaged over frames.
"""

import math

import numpy as np

from .wfs_oracle import pupil_geometry, project


def _star_sensor(theta, lam, D, obs, n_pup):
    """A star at infinity seen on an n_pup x n_pup pupil grid (one subaperture covering it)."""
    return dict(theta_x_rad=float(theta[0]), theta_y_rad=float(theta[1]), src_alt_m=math.inf,
                lambda_m=lam, pupil_d_m=D, obs_d_m=obs, n_sa=1, n_sub=n_pup, n_fft=2 * n_pup,
                bin=1, valid_frac=0.0, na_fwhm_m=0.0, launch_x_m=0.0, launch_y_m=0.0,
                photons=0.0, read_noise_e=0.0)


def science_pupil(D, obs, n_pup):
    """Binary amplitude A [n_pup][n_pup] (the sensors' pupil convention)."""
    return pupil_geometry(_star_sensor((0.0, 0.0), 1.0, D, obs, n_pup))["A"]


def residual_phase(layer_buf, cfg, theta, step, D, obs, n_pup):
    """Phase [n_pup][n_pup] (radians at the reference wavelength) towards direction theta."""
    sensor = _star_sensor(theta, cfg["lambda_ref_m"], D, obs, n_pup)
    return project(np.asarray(layer_buf, dtype=np.float64), cfg, sensor, step)


def psf_frame(phase_ref, A, kappa, N):
    """|DFT(A exp(i kappa phase))|^2 / (N^2 sum A^2), zero-padded to N, zero frequency at
    (N/2, N/2); rows are y frequencies."""
    n = A.shape[0]
    E = np.zeros((N, N), dtype=np.complex128)
    E[:n, :n] = A * np.exp(1j * kappa * phase_ref)
    F = np.fft.fft2(E)
    I = (F.real ** 2 + F.imag ** 2) / (N * N * (A ** 2).sum())
    return np.fft.fftshift(I)


def phase_variance(phase_ref, A, kappa):
    """Piston-removed variance of kappa * phase over the lit pupil (rad^2)."""
    w = A > 0
    p = kappa * phase_ref[w]
    return float((p ** 2).mean() - p.mean() ** 2)


def long_exposure(layer_buf, cfg, stars, steps, lambdas, n_fft, D, obs, n_pup):
    """Summed PSFs {(l, s): [N][N]} and summed phase variances {(l, s): float} over steps."""
    A = science_pupil(D, obs, n_pup)
    psf, var = {}, {}
    for k in steps:
        for s, th in enumerate(stars):
            ph = residual_phase(layer_buf, cfg, th, k, D, obs, n_pup)
            for l, (lam, N) in enumerate(zip(lambdas, n_fft)):
                kap = cfg["lambda_ref_m"] / lam
                psf[l, s] = psf.get((l, s), 0.0) + psf_frame(ph, A, kap, N)
                var[l, s] = var.get((l, s), 0.0) + phase_variance(ph, A, kap)
    return psf, var


def strehl_from_psf(psf_sum, n_frames, A, N):
    """Long-exposure image at zero frequency over the diffraction-limited peak (sum A)^2 /
    (N^2 sum A^2)."""
    peak = A.sum() ** 2 / (N * N * (A ** 2).sum())
    return psf_sum[N // 2, N // 2] / (n_frames * peak)


def strehl_marechal(var_sum, n_frames):
    return math.exp(-var_sum / n_frames)
