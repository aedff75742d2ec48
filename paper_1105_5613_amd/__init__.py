"""MI355X (gfx950) short-range molecular dynamics hot path of arXiv:1105.5613.

The computation lives in ``libmd.so`` (HIP kernels behind the C ABI of
``include/md.h``); ``paper_1105_5613_amd.md`` is the ctypes binding.
"""
from .md import (MD_FP64, MD_MIXED, MD_POT_LJ, MD_POT_SOFT, MD_TRUNC_SHIFT,  # noqa: F401
                 MD_TRUNC_SHIFTED_FORCE, MDError, Params, System, lib, make_params)
