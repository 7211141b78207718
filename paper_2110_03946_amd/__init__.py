"""MI355X-native multilevel ORAS solver for homogeneous diffusion inpainting.

Kaemper & Weickert, "Domain decomposition algorithms for real-time
homogeneous diffusion inpainting in 4K" (arXiv 2110.03946).

The solver is a C-ABI shared library (``include/ddi.h``) of hand-written HIP
kernels for gfx950; ``paper_2110_03946_amd.ddi`` is its thin ctypes binding.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["ddi", "synth"]
