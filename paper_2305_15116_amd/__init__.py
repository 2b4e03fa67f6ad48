"""MI355X-native matrix-free P1 stencils on uniformly refined macro meshes.

The C ABI (include/mf_stencil.h, libmfstencil.so) does all the work in HIP
kernels; this package holds its ctypes binding (same names), the seeded
workload generators and the serving loop.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import EXPORTS, Mesh, MFError, lib  # noqa: F401
