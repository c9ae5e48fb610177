"""Seeded synthetic inputs for the bilateral-filter workloads.

This module only draws and paints test images (piecewise-constant star
polygons, optional smooth gradient, Gaussian noise, integer gray levels) and
the per-image filter parameters of the batched workloads.  It holds none of
the filter's arithmetic, so both the FP64 reference code and the GPU path can
take their inputs from here without sharing any method code.
"""
from .images import (  # noqa: F401
    polygon_image,
    frames,
    batch_specs,
    WORKLOADS,
    workload_images,
    range_table,
)
