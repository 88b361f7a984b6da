"""MI355X Monte Carlo dust radiative transfer (Heymann & Siebenmorgen).

The method runs in the HIP library libmcrt.so behind the C ABI of
include/mcrt.h; this package only marshals arguments to it.
"""
from ._lib import (BW_EPOCH, BW_TICKET, ESCAPED, FROZEN, KILLED, PAH_STOP, McrtError,  # noqa: F401
                   lib)
from .context import RECORD_DTYPE, Context, run_batch, run_opts  # noqa: F401

__all__ = ["Context", "run_batch", "run_opts", "RECORD_DTYPE", "McrtError", "lib", "FROZEN",
           "BW_EPOCH", "BW_TICKET", "ESCAPED", "KILLED", "PAH_STOP"]
