"""MI355X-native Wilson-Clover operator and mixed-precision RAS solver.

The HIP library (``libwcl.so``, built from ``csrc/``) is loaded lazily by
``paper_1612_06556_amd.wcl``; importing the package itself loads nothing.
"""
__all__ = ["synth", "wcl"]
