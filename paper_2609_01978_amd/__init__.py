"""MI355X-native stripe-CZT Fresnel zone plate propagator.

The C ABI (``include/fzp.h``) is implemented by ``libfzp.so`` (HIP, gfx950);
this package is its thin Python binding.  See ``_lib.Plan``.
"""
from ._lib import (FZPError, Graph, MLP, Plan, field_from_log_intensity, log_intensity, load_library, EXPORTED, LIB_PATH, PATH_FP64_BLUESTEIN,  # noqa: F401
                   PATH_SPLIT_BF16, PATH_SA_CZT, grid_for_element, FZP_OK, FZP_E_INVAL, FZP_E_SAMPLING, FZP_E_NOMEM, FZP_E_DEVICE,
                   FZP_E_UNSUPPORTED)

__all__ = ["FZPError", "Graph", "MLP", "Plan", "log_intensity", "field_from_log_intensity", "load_library", "EXPORTED", "LIB_PATH", "PATH_FP64_BLUESTEIN",
           "PATH_SPLIT_BF16", "PATH_SA_CZT", "grid_for_element"]
