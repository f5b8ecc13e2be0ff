"""MI355X-native NNCA-based H2 matrix-vector product.

The computation lives in ``libnnca.so`` (HIP for gfx950, C ABI declared in
``include/nnca.h``); :mod:`paper_2203_14832_amd.nnca` only marshals arguments
to it, and PyTorch supplies device memory and streams.
"""
