"""FP64 CPU oracle for the multibeam transient hot path.

Test infrastructure: only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path never does.
"""
from .ref import *  # noqa: F401,F403
from .ref import (DISPERSION_CONSTANT_S_MHZ2, CANDIDATE_DTYPE, PEAK_DTYPE,  # noqa: F401
                  PlanDesc, RfiParams, RfiResult, NormResult)
