"""MI355X-native solve phase of element-based AMG (AMGe) for lowest-order H(curl) and
H(div) systems: device-resident de Rham hierarchy, hybrid l1-Jacobi smoothing, FP32
V-cycle inside FP64 inexact PCG, all hot operations in hand-written HIP kernels.

Submodules
----------
amge       ctypes binding of libamge.so (the C ABI in include/amge.h)
serve      request mixes for the native serving engine (amge_server_*)
workloads  seeded synthetic inputs (problem sizes, coefficients, right-hand sides)
build      compiles libamge.so for gfx950
"""
__all__ = ["amge", "serve", "workloads", "build"]
