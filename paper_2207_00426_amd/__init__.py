"""Parallel square-root iterated smoothing on MI355X (gfx950).

The compute path is the HIP library ``libpss.so`` (C ABI declared in
``include/pss.h``); :mod:`paper_2207_00426_amd.pss` is its thin Python
binding.  Importing this package does not load the library; the binding
loads it on first use and raises if it is missing.
"""
__all__ = ["workloads", "pss"]
