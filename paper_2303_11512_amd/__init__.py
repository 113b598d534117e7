"""MI355X (gfx950) MG-MLMC++: multigrid multilevel Monte Carlo with Hutch++
deflation for tr(D^{-1}) of the 2D Schwinger operator, as a HIP library with a
C ABI (``include/mgmlmc.h``) and this thin Python binding."""
from ._lib import (  # noqa: F401
    Context,
    MGMError,
    MGParams,
    SolveParams,
    TraceParams,
    TraceResult,
    load_library,
    mg_params,
    solve_params,
    adam_params,
    CNN_NPARAMS,
    PURPOSE_SAMPLE,
    PURPOSE_SETUP,
    PURPOSE_SKETCH,
)
