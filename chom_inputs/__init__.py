"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side callers.

This package holds no arithmetic of the homogenisation method: it only draws the
random workload parameters (temperature, moisture, exposure time and the eight
property factors of each macro Gauss point), states the base material
constants of the plain-weave workload and builds seeded unstructured box
meshes (geometry only).  Everything downstream (degradation law,
stiffness tensors, meshes, solves) is implemented separately by the oracle and by
the HIP library.
"""
from .params import (  # noqa: F401
    BASE_MATERIALS,
    PARAM_FIELDS,
    splitmix64,
    uniform01,
    draw_params,
    draw_factors_only,
    batch_sizes_c2,
    uniform_block,
)
from .umesh import unstructured_box  # noqa: F401
