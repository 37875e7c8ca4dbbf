"""Domain-decomposed ILU0 preconditioning and BiCGSTAB on MI355X (gfx950).

The computation lives in the HIP library libddilu.so (csrc/, C ABI in
include/ddilu.h); ``ddilu`` is its thin ctypes binding and ``solver`` a small
convenience layer that moves a problem's arrays to the device.
"""

from . import ddilu  # noqa: F401
from .ddilu import (  # noqa: F401
    DD_FP32, DD_FP64, DD_MIXED, DDError, Handle, bicgstab_solve, dd_auto_subdims, dd_destroy,
    dd_device_caps, dd_get_factors, dd_get_info, dd_get_levels, dd_get_partition,
    dd_get_reordered, dd_last_error, dd_partition, dd_set_precision, dd_spmv,
    dd_trsv_apply, ilu0_factor,
)
