"""MI355X-native Gaussian molecular surface partition/estimation (after
Liu, Chen & Lu, arXiv:1611.03474).

The numerical path runs in hand-written HIP kernels for gfx950 behind the C
ABI declared in ``include/tms.h``; ``paper_1611_03474_amd.tms`` is the thin
ctypes binding over that library.  Importing this package does not load the
library; the first call into ``tms`` does, and raises if it is missing.
"""

__all__ = ["tms", "synth", "workloads"]
