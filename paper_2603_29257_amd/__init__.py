"""MI355X (gfx950) TDA-risp: factor build and Davidson sigma products as HIP kernels behind a C ABI.

The Python layer only marshals arguments to librisp.so (see include/risp.h); it has no compute
fallback. Build the library first with ``paper_2603_29257_amd.build.build()``.
"""
from .abi import (  # noqa: F401
    BF16, FP32, FP64, PRECISIONS, RSH_COMBINED, RSH_SPLIT, WIN_ABSOLUTE, WIN_FRONTIER, Context, DavInfo,
    Factors, Params, RispError, System, load_library,
)
