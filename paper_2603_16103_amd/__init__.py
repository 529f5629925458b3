"""MI355X (gfx950) implementation of the NanoGS splat-simplification hot path.

The compute lives in ``libnanogs.so`` (HIP kernels behind the C ABI declared
in ``include/nanogs.h``); ``nanogs`` is its Python binding and ``synth`` the
seeded scene generator used by the tests and the benchmark.
"""
