"""MI355X-native dense 3-way MTTKRP and CP-ALS.

The compute path lives in ``libmttkrp.so`` (hand-written HIP for gfx950,
exported through a C ABI declared in ``include/mttkrp.h``).  The Python layer
in :mod:`paper_2411_04785_amd.mttkrp` only marshals arguments; it loads the
library lazily on first use and raises if the library is missing.
"""

__all__ = ["synth"]
