"""kgrt: FP64 Kerr geodesic ray tracing with radiative transfer on MI355X.

Submodules: ``kgrt`` (ctypes binding of the C ABI in include/kgrt.h, needs
torch and the built libkgrt.so), ``scenes`` (seeded synthetic workloads),
``build`` (hipcc build of the library).
"""
