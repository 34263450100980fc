"""Fully edge-weighted personalized PageRank by Monte Carlo walks on MI355X.

The method runs in HIP kernels behind the C-ABI of include/fppr.h
(libfppr.so); `fppr` is its Python binding.
"""
from . import fppr  # noqa: F401
