"""Seeded synthetic inputs for the cylindrical-aperture spherical Radon transform.

This package holds only input generators: sensor sample sets (angles, heights,
radii), voxel grids and phantoms. It contains none of the transform's
arithmetic, so that the HIP path and the FP64 oracle can both consume the same
arrays without sharing any code that computes the method.
"""
from .configs import (Aperture, column_aperture, cylinder_aperture, config, square_columns,  # noqa: F401
                      random_aperture, with_rho_grid, CONFIG_NAMES)
from . import phantoms  # noqa: F401
