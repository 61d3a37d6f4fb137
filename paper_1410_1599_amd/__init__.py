"""MI355X-native multiple-precision matrix multiplication and LU.

Importing the package loads nothing native; ``paper_1410_1599_amd.mp`` holds
the binding of the C-ABI library and loads it on first use.
"""
