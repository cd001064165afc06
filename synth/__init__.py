"""Seeded synthetic catalogs and workload descriptions.

This package only draws random points and describes grids; it holds none of
the correlation arithmetic.  Both the FP64 oracle tests and the HIP path read
the catalogs it produces, so that the two see identical FP32 inputs.
"""
from .catalogs import (  # noqa: F401
    Catalog,
    Workload,
    neyman_scott_box,
    uniform_box,
    neyman_scott_cap,
    uniform_cap,
    lognormal_weights,
    workload,
    WORKLOADS,
    mock_catalog,
    mock_sizes,
    MOCK_RADII,
)
