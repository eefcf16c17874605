"""MI355X (gfx950) TDA-risp: factor build and Davidson sigma products as HIP kernels behind a C ABI.

The Python layer only marshals arguments to librisp.so (see include/risp.h); it has no compute
fallback. Build the library first with ``paper_2603_29257_amd.build.build()``; the binding is
loaded on first use of a name below, so the build module imports without the library.
"""
_EXPORTS = ("BF16", "FP32", "FP64", "PRECISIONS", "RSH_COMBINED", "RSH_SPLIT", "WIN_ABSOLUTE",
            "WIN_FRONTIER", "Context", "DavInfo", "Factors", "Params", "RispError", "System", "load_library",
            "PHASES", "job_footprint", "J_MO", "J_AO_DIRECT", "device_usage")


def __getattr__(name):
    if name in _EXPORTS:
        from . import abi
        return getattr(abi, name)
    raise AttributeError(name)


__all__ = list(_EXPORTS)
