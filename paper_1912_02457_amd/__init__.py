"""MI355X (gfx950) implementation of the eta-based, well-balanced
central-upwind shallow-water scheme of Brodtkorb & Holm (arXiv 1912.02457).

The scheme runs in hand-written HIP kernels behind the C ABI of
``include/swe.h``; ``swe`` is its thin ctypes binding.  The HIP library must
be built (``paper_1912_02457_amd.build.build()``): using a domain without it
raises ImportError, there is no CPU fallback.
"""

from .swe import (  # noqa: F401
    BC_NESTED, BC_PERIODIC, BC_WALL, FRICTION_LINEAR, FRICTION_MANNING, FRICTION_NONE,
    FRICTION_QUADRATIC, LIB_PATH, Domain, Ensemble, Params, Server, SweError, coarsen2, erode_land,
    load_library, make_params, reconstruct_bathymetry, refine2, workspace_bytes,
)
