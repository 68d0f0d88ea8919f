"""FP64 CPU oracle for the unsplit wave-propagation step of 2D acoustics.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and the two share no code.
"""

from .oracle import (  # noqa: F401
    BC,
    LIM,
    adjoint_run,
    adjoint_step,
    build,
    conservation_sums,
    fill_bc,
    forward_traces,
    frozen_step,
    lib,
    mc_branch,
    phi,
    riemann_edge,
    run,
    split_vec,
    step,
    step_patches,
)
