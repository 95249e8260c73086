"""MI355X-native block-iterative CT reconstruction (CSGD / GCSGD).

The solver lives in the HIP library ``libctcsgd.so`` behind the C ABI of
``include/ct.h``; ``paper_1709_00953_amd.ct`` is its Python binding and
``paper_1709_00953_amd.inputs`` builds seeded synthetic workloads.
Importing the package loads nothing.
"""
