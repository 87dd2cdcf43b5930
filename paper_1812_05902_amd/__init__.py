"""MI355X-native ray-traced synthetic PIV/BOS image generation.

The compute path is the C-ABI library ``libpbr.so`` (hand-written HIP kernels for gfx950,
declared in ``include/pbr.h``); ``paper_1812_05902_amd.pbr`` is its thin Python binding and
``paper_1812_05902_amd.inputs`` holds the seeded synthetic scenes.  Importing this package
loads nothing native; the binding loads the library on first use and fails loudly if it has
not been built.
"""
__all__ = ["inputs", "pbr"]
