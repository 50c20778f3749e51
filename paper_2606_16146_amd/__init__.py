"""MI355X (gfx950) SumCheck prover for multilinear ZeroCheck over BN254 Fr.

The compute runs in the HIP library ``libzc.so`` (C ABI in include/zc.h);
``zc`` is its Python binding.  Importing this package loads nothing.
"""
