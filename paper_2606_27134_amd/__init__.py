"""libdmkloc: leaf-level residual interaction of the periodized DMK method
on AMD MI355X (gfx950).

The compute path is the HIP library ``libdmkloc.so`` (C ABI in
``include/dmk.h``); this package holds its ctypes binding
(:mod:`._lib`), PyTorch-facing wrappers and the autograd function
(:mod:`.residual`), the build script (:mod:`.build`) and the seeded input
generators (:mod:`.workloads`).  Importing the package loads nothing; the
library is loaded on first use.
"""
__all__ = ["residual", "workloads", "build"]
