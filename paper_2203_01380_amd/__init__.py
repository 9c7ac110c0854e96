"""MI355X (gfx950) diffusive integer lattice gas with the flip operator.

The compute path lives in libilg.so (HIP kernels behind the C ABI of
include/ilg.h); this package is its thin Python binding.  Importing the
binding requires the built library: there is no CPU fallback.
"""
from ._ilg import (ABI_VERSION, MAX_K, IlgError, Lattice, binomial_table, fixed_point,  # noqa: F401
                   lib, make_config)
