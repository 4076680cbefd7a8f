"""Correctly rounded elementwise math for AMD Instinct MI355X (gfx950).

The compute path is the HIP library libcr.so (C ABI in include/cr.h); the
Python module `crmath` is a ctypes binding of it and `inputs` holds the
seeded synthetic workload generators.
"""
