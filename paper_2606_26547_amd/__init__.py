"""MI355X-native HDC classification hot path (random-projection encoding,
majority bundling, Hamming-distance argmin, approximation knobs).

The compute path lives in the HIP/C-ABI library ``libhdc.so`` built from
``csrc/``; ``hdc`` is its thin Python binding.  Importing this package does
not load the library; ``paper_2606_26547_amd.hdc`` does, and raises if it
has not been built.
"""
__all__ = ["datagen", "hdc"]
