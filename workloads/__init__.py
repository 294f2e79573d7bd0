"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *generates inputs*: simplicial meshes, overlay-grid
descriptions, right-hand-side samples and random vectors.  It holds none of
the grid-overlay method's arithmetic (no transfer weights, no Toeplitz
coefficients, no operator applications), so both the CPU oracle and the HIP
library can consume its output without sharing any of the method's code.
"""

from .meshes import (  # noqa: F401
    Mesh,
    disk_mesh,
    interval_mesh,
    lshape_mesh,
    star_mesh,
    ball_mesh,
    structured_box_mesh,
    structured_box_mesh_3d,
    star_radius_fn,
)
from .grids import Grid, grid_for_box, grid_node_coords_1d  # noqa: F401
from .rhs import fourier_rhs, constant_rhs, eval_fourier  # noqa: F401
from .configs import config_inputs  # noqa: F401
