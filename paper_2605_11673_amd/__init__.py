"""Exact streaming assembly of A_t = M_t + dt^2 K_t on MI355X (gfx950).

The GPU path lives in ``csrc/`` (HIP kernels and a C ABI, ``libstafem.so``);
``stafem`` is its thin Python binding and ``workloads`` the seeded input
generators.  Importing the package does not load the GPU library: the
binding loads it on first use and raises if it is missing.
"""
__all__ = ["workloads", "stafem"]
