"""MI355X-native light-field renderer: the interleaved image of a slanted-lenticular panel rendered
directly from a 3D Gaussian splatting scene (DirectL, arXiv 2407.14053), on hand-written gfx950 kernels
behind a C ABI (``include/directl.h``).

The HIP library is loaded lazily on first use (``paper_2407_14053_amd.api``); importing the package does not
touch the GPU.  ``synth`` draws the seeded synthetic inputs.
"""
__all__ = ["api", "synth"]
