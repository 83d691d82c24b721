"""MI355X (gfx950) moving-least-squares field library.

Evaluates the moving-least-squares interpolation of Muelder et al. (Sec. 3.3,
Eq. 4-8) on a grid over scattered points with D attributes, in hand-written
HIP kernels behind a C ABI (include/mls.h).  The Python layer only marshals
arguments: see :mod:`paper_1408_0677_amd.api`.
"""
from .api import (BASIS, PRECISION, WEIGHT, MlsError, Context, Server, ServerError,  # noqa: F401
                  contour, fit, fit_scratch_bytes)
