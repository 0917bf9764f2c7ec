"""MI355X-native line-by-line Monte-Carlo radiative ray tracer (HIP, gfx950).

Importing the package loads nothing; ``paper_cs_0703028_amd.rtlbl`` binds the
C-ABI library ``librtlbl.so`` built from ``csrc/``.
"""
__all__ = ["inputs", "rtlbl"]
