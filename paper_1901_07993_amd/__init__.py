"""MI355X (gfx950) inverse factorization: iterative refinement (IRSI) and
localized inverse factorization (LIF) on block-sparse matrices, behind the C
ABI of include/lif.h.  ``lif`` is the ctypes binding; ``build`` compiles the
HIP library in-tree."""
from .lif import (  # noqa: F401
    Factorization, LifError, load, HostBlocks,
    FP64, MIXED_FP32, MIXED_BF16, STOP_PAPER, STOP_TOL,
    START_SQRT2_OVER_GERSH, START_INV_SQRT_GERSH, START_INV_SQRT_LMAX, START_GIVEN,
)
