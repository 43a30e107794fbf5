"""MI355X-native primal hybrid FEM hot path (arXiv:2401.15557).

The compute path is the HIP library ``libphfem.so`` behind the C ABI declared
in ``include/phfem.h``; ``paper_2401_15557_amd.phfem`` is its thin ctypes
binding and ``paper_2401_15557_amd.meshgen`` builds seeded synthetic meshes.
Importing this package loads nothing; the library is loaded on first use.
"""
