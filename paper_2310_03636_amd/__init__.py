"""MI355X-native spin-1 split-step library (hand-written HIP for gfx950).

The product path is ``libspin1.so`` (C ABI, include/spin1.h) and its thin
ctypes binding ``paper_2310_03636_amd.spin1``.
"""
