"""MI355X (gfx950) hot path of the frequency/time hybrid wave-equation solver
(Anderson, Bruno & Lyon, arXiv 1807.02718, Part I).

The compute lives in libfhw.so (HIP kernels behind the C ABI in
include/fhw.h); `paper_1807_02718_amd.fhw` is its ctypes binding.
"""
__all__ = ["fhw", "build"]
