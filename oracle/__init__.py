"""FP64 CPU oracle of the Shack-Hartmann wavefront-sensor path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The product library (``paper_1608_00386_amd``) never imports, links or
calls anything here, and this package imports nothing from it: the two share no code, only the
seeded inputs of ``synth/``.

The oracle is a plain, slow, obviously correct numpy FP64 implementation of what the path
computes, step by step in the order of the paper's closed-loop description (Sec. 2.2 open-loop
wavefront by geometric projection, Sec. 2.7 X/Y slopes from the residual phase, slopes times
the control matrix, integrator), with the sensor internals (zero-padded subaperture FFT,
sodium elongation, binning, noise, centre of gravity) that the paper leaves unspecified taken
from the readings listed in the design notes.  Parity of functions whose result the paper does
not fix numerically is pinned by closed forms, invariants and brute force in ``tests/``.
"""

from .wfs_oracle import (  # noqa: F401
    pupil_geometry,
    subap_centres,
    project,
    project_transpose,
    subap_fields,
    spots,
    elongation_kernel,
    elongate,
    bin_spots,
    add_noise,
    noise_normals,
    flux,
    centroid,
    sensor_slopes,
    forward,
    adjoint,
    loss,
    recon,
    closed_loop_step,
    n_slopes,
    pixel_scale,
)
from .calib_oracle import interaction_matrix, reference_slopes, regularised_lse  # noqa: F401,E501
from .psf_oracle import (  # noqa: F401
    science_pupil, residual_phase, psf_frame, phase_variance, long_exposure, strehl_from_psf,
    strehl_marechal)
from .screen_oracle import (  # noqa: F401
    screen_normals, von_karman_psd, screen_spectrum, phase_screen)
from .philox import philox4x32_10, philox4x32_10_scalar, uniforms_from_words  # noqa: F401
