"""Seeded synthetic inputs (scanner geometry, spectra, attenuation stand-in,
phantoms, Poisson measurements) shared by the tests, the oracle checks and the
benchmark.  Nothing in this package implements the reconstruction method."""
from .geometry import Geometry, FAN2D, HELICAL3D, ray_endpoints  # noqa: F401
from .configs import (make_inputs, geometry_for, blob_inputs, unrolled_inputs,  # noqa: F401
                      WORKLOADS, PENALTY, mar_params, phantom_for, bowtie)
