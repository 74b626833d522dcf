"""Ozaki-scheme density-matrix purification for AMD MI355X (gfx950).

The computation lives in the HIP library ``libdmp.so`` (see ``include/dmp.h``);
``api`` is its thin torch binding.  Importing this package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from ._lib import DmpError  # noqa: F401
from .api import (Purify, PurifyTape, autotune_slices, max_slices, ozaki_gemm,  # noqa: F401
                  ozaki_gemm_noalloc,
                  ozaki_gemm_batched, purify, purify_batched, version)
