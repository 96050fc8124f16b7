"""MI355X-native destriping of CMB polarimeter timelines (arXiv:1309.5609 hot path).

The computation lives in ``libdst.so`` (HIP for gfx950, C ABI in
``include/dst.h``); ``paper_1309_5609_amd.dst`` is its thin Python binding.
"""
from .dst import (Context, DstError, Problem, dst_apply_operator, dst_baseline_reduce, dst_bin,  # noqa: F401
                  dst_pixel_setup, dst_residual, dst_solve, dst_unbin, library, to_device)
