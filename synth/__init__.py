"""Seeded synthetic inputs for NAO real-space grid integration.

The package only *constructs inputs*: geometries, analytic radial tables on the logarithmic
knot grid, atom-centred integration grids with partition weights, the potential on the grid and
the density matrix.  It performs none of the integration arithmetic (no spline interpolation,
no spherical harmonics, no contractions), so both the FP64 oracle and the HIP library can
consume its output without sharing any of the method's code.
"""
from .instances import (  # noqa: F401
    Instance,
    CONFIGS,
    make_instance,
    make_molecule_set,
    regrid,
    radial_shells,
    generator_device,
    custom_instance,
    becke_radial,
    angular_gauss_legendre,
    angular_lobatto,
    stratmann_partition,
    radial_tables,
    log_knots,
)
