"""MI355X-native finite-volume hot path (arXiv:1912.07645, Section 2): libfv.so, a C-ABI
library of hand-written HIP kernels for gfx950, and a thin Python binding.

``paper_1912_07645_amd.fv`` holds the C names (fv_create, fv_evolve, fv_stats_accumulate,
...); ``Solver`` and ``Stats`` wrap them with torch tensors for device memory. The library is
loaded on first use of any of these names and raises ImportError if libfv.so is missing
(there is no CPU fallback); ``paper_1912_07645_amd.build`` compiles it.
"""
import importlib

__all__ = ["fv", "Solver", "Stats", "evolve_multi", "mlmc_combine"]


def __getattr__(name):
    if name == "fv":
        return importlib.import_module(".fv", __name__)
    if name in ("Solver", "Stats", "evolve_multi", "mlmc_combine"):
        return getattr(importlib.import_module(".solver", __name__), name)
    raise AttributeError(name)
