"""MI355X-native short-range non-bonded force path (cell list, cutoff filter,
Lennard-Jones 12-6 + switched Coulomb) behind a C ABI.

Importing the package loads nothing; ``paper_1611_04474_amd.api`` loads the HIP
library on first use and fails loudly if it is missing.
"""
__all__ = ["workloads", "api"]
