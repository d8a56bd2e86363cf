"""MI355X-native ConeGaussian renderer: per-pixel anti-aliased Gaussian ray rendering
for generic central cameras (HIP kernels for gfx950 behind a C ABI).

Importing the package loads nothing native; ``paper_2609_13397_amd.render`` loads
the HIP library on first use and raises if it is missing.
"""
__all__ = ["synth"]
