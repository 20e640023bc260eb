"""MI355X Shack-Hartmann wavefront-sensor path (projection, spots, elongation, binning, noise,
centroids, reconstructor) as hand-written HIP kernels behind the C ABI of include/wfs.h."""

from ._lib import (  # noqa: F401
    WFS_FLAG_ADJOINT_ATOMIC,
    WFS_FLAG_FORCE_FFT,
    WFS_FLAG_FUSED,
    WFS_FLAG_FOOTPRINT,
    WFS_FLAG_FORCE_OTF,
    WFS_FLAG_NO_XCD_REMAP,
    WFS_FLAG_SPLIT,
    WFS_STEP_DEVICE,
    WfsError,
    lib,
)
from .wfs import Plan, WFSFunction, recon_apply, tlse, wfs_slopes  # noqa: F401
from . import calib  # noqa: F401
from .psf import PsfPlan, screen_generate  # noqa: F401
