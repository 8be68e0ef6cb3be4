"""MI355X-native hot path of pixel-level distributed 3D Gaussian splatting
(Splaxel, arXiv 2606.18588): HIP kernels for gfx950 behind the C ABI of
libsplaxel.so (include/splaxel.h), with a thin Python binding.

Importing the package does not load the library; ``binding.lib()`` does, and
raises if it has not been built (``python -m paper_2606_18588_amd.build``).
"""
__all__ = ["binding", "pipeline", "build"]
