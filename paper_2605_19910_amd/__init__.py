"""MI355X-native recursive Green's function (RGF / DDRGF) selected inversion.

The computation lives in the HIP library ``lib/librgf.so`` (C ABI in
``include/rgf.h``); :mod:`paper_2605_19910_amd.binding` marshals torch tensors to
it.  Importing this package does not load the library; the first call does, and it
fails loudly when the library has not been built.
"""
from .binding import (BatchedPlan, Plan, RgfError, device_table, load, rgf_batched_solve,  # noqa: F401
                      solve, solve_batched)

__all__ = ["BatchedPlan", "Plan", "RgfError", "device_table", "load", "rgf_batched_solve", "solve",
           "solve_batched"]
