"""MI355X-native solver for Inductive Convolution Nuclear Norm Minimization (ICNNM).

The solver lives in the HIP library ``libicnnm.so`` (C ABI in include/icnnm.h);
``paper_2604_17001_amd.icnnm`` is its Python binding and
``paper_2604_17001_amd.inputs`` draws seeded synthetic problems.
"""
__all__ = ["icnnm", "inputs", "build"]
