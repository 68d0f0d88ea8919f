"""MI355X-native unsplit wave-propagation step for 2D linear acoustics on
batched AMR patches (after Qin, LeVeque & Motley, arXiv 1808.02638).

The computation lives in the gfx950 HIP library ``libwavestep.so`` behind the
C ABI of ``include/wavestep.h``; this package marshals arguments to it and uses
PyTorch for device memory and streams only.
"""

from ._lib import WaveStepError  # noqa: F401
from .level import Level  # noqa: F401
from .adjoint import AcousticsAdjoint  # noqa: F401
from .amr import Hierarchy, TwoLevel  # noqa: F401
