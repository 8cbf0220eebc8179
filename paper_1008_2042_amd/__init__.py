"""Tight-frame regularised cone-beam CT reconstruction on MI355X (gfx950).

The compute path is the HIP library ``libtfcb.so`` behind the C-ABI declared
in ``include/tfcb.h``; ``paper_1008_2042_amd.tfcb`` is its thin Python
binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["inputs", "tfcb"]
