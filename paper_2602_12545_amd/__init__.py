"""MI355X implicit flux-limited-diffusion radiation step (HIP, gfx950).

Thin Python layer over the C ABI of libfld.so (include/fld.h); the entry
points keep their C names (fld_create, fld_assemble, fld_solve, fld_step,
fld_steps, fld_get_operator, fld_destroy; fld_batch_*; fld_forest_*) on ``lib``
and are wrapped by ``Context``, ``Batch`` and ``Forest``.  Importing fails if the HIP library has not been built.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import Batch, Context, FLDError, Forest, default_options, lib, LIB_PATH  # noqa: F401
