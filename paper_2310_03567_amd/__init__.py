"""MI355X-native incremental octree LOD insertion (SimLOD, arXiv 2310.03567).

The work runs in hand-written gfx950 HIP kernels behind the C ABI in
include/simlod.h (libsimlod.so, built in-tree); ``simlod`` is its ctypes
binding.  Importing ``paper_2310_03567_amd.simlod`` fails if the library is
not built.
"""

__all__ = ["simlod"]
