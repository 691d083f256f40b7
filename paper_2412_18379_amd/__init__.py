"""MI355X-native CNN-SNS particle location (arXiv 2412.18379) on 2D triangle meshes.

The computation lives in libcnnsns.so (HIP for gfx950, C ABI in
include/cnnsns.h); ``cnnsns`` is its ctypes binding, ``workload`` the seeded
synthetic input generator.  Import those submodules explicitly.
"""
__all__ = ["cnnsns", "workload", "build"]
