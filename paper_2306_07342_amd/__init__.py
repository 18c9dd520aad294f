"""MI355X-native density-matrix emulation core (arXiv 2306.07342, VQD).

The compute path is the HIP library ``libvqd.so`` (C ABI in include/vqd.h);
:mod:`paper_2306_07342_amd.vqd` is its thin Python binding.
"""
__all__ = ["vqd"]
