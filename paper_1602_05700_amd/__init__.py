"""MI355X-native hyperbolic self-gravity solver (arXiv:1602.05700).

The compute path is the HIP library ``libhgs.so`` (C ABI in include/hgs.h);
``paper_1602_05700_amd.hgs`` is its Python binding.
"""
__all__ = ["hgs"]
