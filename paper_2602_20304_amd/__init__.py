"""MI355X (gfx950) smooth contact-manifold generation.

The compute path lives in libcm.so (HIP kernels + C ABI, include/cm.h);
``paper_2602_20304_amd.cm`` is the Python binding.  Importing the package does
not load the library; ``cm.Context`` does, and raises if it is missing.
"""
__all__ = ["cm", "build", "opmodel"]
