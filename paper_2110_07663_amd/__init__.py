"""MI355X-native spectral-element Poisson solver (arXiv:2110.07663 hot path).

The compute path lives in the HIP/C++ shared library built from csrc/ (C ABI
declared in include/sem.h); `sem` is its thin ctypes binding and `workloads`
holds the seeded synthetic inputs.  Importing this package does not load the
library: `sem.lib()` does, and raises if it is missing.
"""
__all__ = ["sem", "workloads"]
