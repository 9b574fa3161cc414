"""MI355X-native Galerkin assembly for the IgA-SGBEM (2D Laplace single-layer
operator, periodic B-splines on closed curves): B-spline weighted quadrature
with row assembly and sum factorisation, element-by-element Gauss assembly,
right-hand side and mixed-precision solve, as hand-written HIP kernels for
gfx950 behind the C ABI of include/sgbem.h.

``paper_1703_10016_amd.sgbem`` is the ctypes binding (same names as the C
ABI); ``paper_1703_10016_amd.runtime`` wraps it with torch device memory.
"""
