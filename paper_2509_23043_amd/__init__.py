"""MI355X (gfx950) implementation of the TAPT hot path (arXiv:2509.23043).

``binding`` exposes libtapt.so (HIP kernels behind the C ABI of
include/tapt.h); ``inputs`` generates seeded synthetic problems.
"""
