"""Cyclic compact-banded solves by parallel cyclic reduction on MI355X (gfx950).

The compute path is the C-ABI library `libcb.so` (hand-written HIP kernels);
`paper_2101_02286_amd.cb` is its thin Python binding.  Importing the package
does not load the library; `cb` loads it on first use and raises if it is
missing.
"""
__all__ = ["cb", "synth"]
