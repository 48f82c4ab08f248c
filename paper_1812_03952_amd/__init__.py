"""MI355X-native CPR-GMRES linear solve of a fully implicit thermal reservoir
simulator (Liu & Chen, arXiv 1812.03952): librsolve.so (HIP kernels for
gfx950 behind a C-ABI, see include/rsolve.h) and its Python binding."""
from . import rsolve  # noqa: F401
