"""Restricted additive Vanka (RAV) geometric multigrid for Taylor-Hood Q2/Q1
Stokes systems on MI355X (gfx950).

The numerical work lives in ``librav.so`` (HIP kernels behind the C-ABI of
``include/rav.h``); :mod:`paper_2103_10127_amd.capi` is its ctypes binding.
"""
from .capi import Hierarchy, RavError, lib, stream_copy  # noqa: F401
