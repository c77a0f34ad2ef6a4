"""lcemd on MI355X: RWMD / OMR / ACT / ICT lower bounds of the Earth Mover's
Distance for a query batch against a resident CSR histogram database
(Atasu & Mittelholzer, ICML 2019), computed by hand-written HIP kernels for
gfx950 behind a C ABI (include/lcemd.h).  ``lcemd`` is the ctypes binding."""
from .lcemd import (  # noqa: F401
    Context,
    LcemdError,
    load_library,
    open_context,
)
