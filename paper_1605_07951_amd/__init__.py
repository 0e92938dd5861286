"""MI355X-native resolvent sampling (RSRR hot path): HIP library + thin binding.

The binding (``paper_1605_07951_amd.rsrr``) loads ``librsrr.so`` lazily on first
use and raises if it has not been built.
"""
__all__ = ["rsrr"]
