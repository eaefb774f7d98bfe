"""Near-circulant splitting (NCS) for TV-regularised CT and PET on MI355X (gfx950).

The solver is the C-ABI library ``libncs.so`` (declared in ``include/ncs.h``);
``paper_1810_13100_amd.ncs`` is its Python binding.
"""
from .ncs import (  # noqa: F401
    DATA_POISSON, DATA_QUADRATIC, NCS_ERR_DIVERGED, NCS_ERR_INVALID_ARG, NCS_ERR_NONFINITE,
    NCS_NOT_CONVERGED, NCS_OK, TV_ANISO, TV_ISO, Geometry, NcsError, Params, Solver, load_library,
)
