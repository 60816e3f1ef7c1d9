"""k-input RNS-CKKS ciphertext multiplication on MI355X (gfx950).

``mick`` is the Python binding of the C-ABI library ``libmick.so`` (built by
``build.py`` from ``csrc/``); PyTorch supplies device memory and streams.
"""
