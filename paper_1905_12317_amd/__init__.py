"""MI355X (gfx950) implementation of the FTK rigid-alignment hot path.

The computation lives in libftk.so (HIP kernels + C-ABI, include/ftk.h);
`ftk` is its thin ctypes binding.
"""
from . import ftk  # noqa: F401
from .ftk import MLP, Batch, Plan, ftk_plan_tables, poses_numpy  # noqa: F401
