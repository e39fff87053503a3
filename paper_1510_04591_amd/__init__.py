"""MI355X (gfx950) accelerated divide-and-conquer symmetric tridiagonal eigensolver.

The solver is libadc.so (HIP kernels behind the C ABI in include/adc.h);
`paper_1510_04591_amd.adc` is its ctypes binding and `workloads` holds the
seeded synthetic inputs.  Importing this package loads nothing: the library
is opened on first use.
"""
__all__ = ["adc", "workloads"]
