"""MI355X-native UniFrac distances (striped and matrix-core hot paths in HIP for gfx950).

The compute lives in libunifrac_mi.so (C ABI: include/unifrac_mi.h); this package is its
thin Python binding.  Importing it loads the library and fails if it has not been built.
"""
from .binding import (  # noqa: F401
    Batch,
    Context,
    EXPORTED,
    LIB_PATH,
    METHODS,
    PRECISIONS,
    Plan,
    UfTuning,
    UniFracError,
    distance,
    distance_batch,
    library,
    mantel,
    merge_block,
    validate,
    validate_problem,
)
