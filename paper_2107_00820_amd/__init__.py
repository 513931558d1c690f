"""stk: augmented-Lagrangian Stokes multigrid on AMD MI355X (gfx950).

The compute path is libstk.so (hand-written HIP kernels behind the C ABI in
include/stk.h); ``paper_2107_00820_amd.stk`` is its ctypes binding. The
library is loaded lazily on first use and the binding raises if it is
missing; nothing here falls back to a CPU implementation.
"""
from .stk import (Hierarchy, StkError, load, make_desc, desc_from_workload, stk_footprint, stk_step_batch,  # noqa: F401
                  STK_OK, STK_EINVAL, STK_ENOMEM, STK_EDEVICE, STK_ENOTCONV, STK_ENOTSPD, STK_ENAN,
                  STK_EBUSY, STK_F64, STK_F32)
