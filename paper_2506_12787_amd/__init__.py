"""SwiftWRF render path for MI355X (gfx950): deformation MLP, preprocess,
scan + radix sort, tile blending, backward and serving, behind a C ABI
(libswiftwrf.so). Importing the package loads nothing; the native library is
loaded on first use by `paper_2506_12787_amd.binding`.
"""
__all__ = ["synth", "binding"]
