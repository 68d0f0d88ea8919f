"""Seeded synthetic inputs for the acoustics wave-propagation workloads.

This module only builds inputs: grids, patch layouts, initial conditions,
material parameters and receiver positions.  It holds none of the numerical
method's arithmetic, and it is shared by the tests, the benchmark and the
library's users alike.
"""

from .generators import (  # noqa: F401
    AMR_LEVEL3_HALF_WIDTH,
    AdjointSetup,
    EnsembleInstance,
    PatchSpec,
    adjoint_setup,
    amr_level_batch,
    ensemble,
    layered_medium,
    padded_centres,
    padded_state,
    plane_wave_state,
    radial_pulse,
    three_level_layout,
    two_level_layout,
    uniform_patch,
)
