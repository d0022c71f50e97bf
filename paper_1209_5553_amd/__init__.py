"""MI355X-native exponential Rosenbrock-Euler (EREM) heat-transport path.

The computation lives in liberem.so (HIP kernels for gfx950 behind the C ABI
of include/erem.h); ``api`` is a thin torch binding and ``inputs`` holds the
seeded synthetic workloads.
"""
__all__ = ["api", "inputs", "build"]
