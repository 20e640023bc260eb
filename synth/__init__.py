"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds the workload *parameters* (telescope, guide stars, turbulence layers,
deformable-mirror grids) and the seeded generators of the *inputs* (von Karman phase screens,
the random reconstructor).  It holds none of the wavefront-sensor arithmetic: projection,
spots, elongation, binning, noise and centroiding live separately in ``oracle/`` (CPU, FP64)
and in ``paper_1608_00386_amd`` (HIP), which share no code.
"""

from .configs import (  # noqa: F401
    LAMBDA_REF_M,
    DT_S,
    config0,
    config1,
    config2,
    config3,
    config4,
    small_lgs,
    layer_offsets,
)
from .screens import (  # noqa: F401
    von_karman_screen,
    make_layers,
    make_batch,
    make_reconstructor,
    random_field,
)
