"""MI355X-native convective right-hand side of a multicomponent compressible
flow solver (XFluids, arXiv 2403.05910): Roe-averaged characteristic WENO5-JS
with LLF splitting, flux divergence, Newton temperature recovery and SSP-RK3,
as hand-written HIP kernels behind a C ABI (``include/xf.h``).

Submodules:
  workloads  seeded synthetic inputs (thermo tables, initial conditions)
  xf         ctypes binding of libxf.so plus torch-facing helpers
"""
