"""MI355X (gfx950) Schur-complement + PCG solver for the LQ subproblem of an NMPC step.

The compute path is the HIP library ``libmpcpcg.so`` (C ABI in include/mpcpcg.h); this
package only marshals torch device tensors into it.  ``synth`` draws seeded problems.
"""
from .mpcpcg import (BREAKDOWN, NOT_CONVERGED, OK, TIMEOUT, Context, MPCPCGFunction,  # noqa: F401
                     load_library)
