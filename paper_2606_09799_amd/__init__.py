"""MI355X (gfx950) implementation of the per-time-step hot path of the
sharp-interface immersed boundary fractional-step scheme (Vagnoli,
Scarpolini, Verzicco, Viola): tagging, two-sided forcing, approximate-
factorisation viscous solves, consistent mass correction and the
FFT/tridiagonal Poisson solve, as hand-written HIP kernels behind the C-ABI
of include/ibm.h.

`paper_2606_09799_amd.ibm` is the ctypes binding of libibm.so (built by
`python -m paper_2606_09799_amd.build`); it raises on import when the library
is missing.
"""
