"""MI355X (gfx950) diffusive integer lattice gas with the flip operator.

The compute path lives in libilg.so (HIP kernels behind the C ABI of
include/ilg.h); this package is its thin Python binding.  Importing the
binding requires the built library: there is no CPU fallback.
"""
from ._ilg import (ABI_VERSION, BATCH_MAX_K, MAX_K, Batch, IlgError, Lattice,  # noqa: F401
                   Server, binomial_table, fixed_point, lib, make_config, probe_philox,
                   probe_stream)
