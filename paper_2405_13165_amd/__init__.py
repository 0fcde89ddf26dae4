"""MI355X (gfx950) library for the meshfree GFDM hot path of "Adaptive coupling
of 3D and 2D fluid flow models": neighbourhoods, local PCA transition
detection, second-order GFDM stencils, stencil application, the pressure
Poisson solve, the 3D->2D transition and adjoints.

The compute path is the HIP library libgfdm.so (C ABI in include/gfdm.h);
`paper_2405_13165_amd.gfdm` is its Python binding.  Importing this package
does not load the library; `gfdm.load_library()` does, and fails loudly if it
has not been built.
"""
__all__ = ["gfdm", "workloads", "build"]
