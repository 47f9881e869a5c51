"""Multi-resolution screen-space lighting on AMD MI355X (gfx950).

Besenthal, Maisch, Ropinski, "Multi-Resolution Rendering for Computationally
Expensive Lighting Effects" (arXiv 1906.04576): edge detection, mask pyramid,
masked per-level lighting (SSAO, PCSS soft shadows, SSGI) and
upsample-and-merge, as hand-written HIP kernels behind the C ABI of
include/mr.h.  ``mr`` is the ctypes binding; ``build`` compiles libmr.so.
"""
from . import mr  # noqa: F401
