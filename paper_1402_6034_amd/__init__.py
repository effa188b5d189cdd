"""MI355X-native round-off DCT (RDCT) hot path: HIP kernels behind a C-ABI library.

Importing the package loads nothing; `paper_1402_6034_amd.rdct` loads the HIP
library and fails loudly when it is missing.
"""
__all__ = ["rdct", "synth"]
