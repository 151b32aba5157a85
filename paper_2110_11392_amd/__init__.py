"""MI355X-native near-field force of the Abacus N-body method.

The HIP library (``libabacus_nf.so``, C ABI in ``include/abacus_nf.h``) is loaded
on first use of ``NearField`` / ``near_field``; importing the package itself
needs no GPU.
"""
from .nearfield import (ACCUMULATION, LAWS, PRECISIONS, Binned, BoxSpec, NearField, near_field,
                        timestep, timing_enable, timing_read, timing_reset)

__all__ = ["ACCUMULATION", "LAWS", "PRECISIONS", "Binned", "BoxSpec", "NearField", "near_field",
           "timestep", "timing_enable", "timing_read", "timing_reset"]
