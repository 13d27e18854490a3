"""MI355X-native restarted narrow-band fast marching (Yang & Stern, arXiv 1502.07303).

The solver itself lives in the HIP library ``libfmm.so`` (sources under
``csrc/``, C ABI in ``include/fmm.h``); ``fmm`` is its Python binding and
``inputs`` builds seeded synthetic workloads.
"""
__all__ = ["fmm", "inputs"]
